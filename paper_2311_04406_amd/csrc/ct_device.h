// ct_device.h -- device-side arithmetic of Z_{2^128}, the counter-based
// generator and the wavefront reductions used by every kernel.
#pragma once

#include "ct_internal.h"

namespace ct {

// ---------------------------------------------------------------- Z_{2^128}

__device__ __forceinline__ u128 mk(uint64_t lo, uint64_t hi) { return u128{lo, hi}; }
__device__ __forceinline__ u128 zero128() { return u128{0, 0}; }

__device__ __forceinline__ u128 add(u128 a, u128 b) {
    u128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
    return r;
}
__device__ __forceinline__ u128 sub(u128 a, u128 b) {
    u128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1ull : 0ull);
    return r;
}
// a * b mod 2^128
__device__ __forceinline__ u128 mul(u128 a, u128 b) {
    u128 r;
    r.lo = a.lo * b.lo;
    r.hi = __umul64hi(a.lo, b.lo) + a.lo * b.hi + a.hi * b.lo;
    return r;
}
// a * b mod 2^128 for a 64-bit b
__device__ __forceinline__ u128 mul64(u128 a, uint64_t b) {
    u128 r;
    r.lo = a.lo * b;
    r.hi = __umul64hi(a.lo, b) + a.hi * b;
    return r;
}
// acc + a * b (b 64-bit)
__device__ __forceinline__ u128 mad64(u128 acc, u128 a, uint64_t b) { return add(acc, mul64(a, b)); }
__device__ __forceinline__ u128 mad(u128 acc, u128 a, u128 b) { return add(acc, mul(a, b)); }

__device__ __forceinline__ u128 ld(const u128 *p, int64_t i) {
    const ulonglong2 v = reinterpret_cast<const ulonglong2 *>(p)[i];
    return u128{v.x, v.y};
}
// A load of streamed data that is not read again soon (non-temporal hint:
// it does not displace reused lines from the caches).
__device__ __forceinline__ u128 ld_nt(const u128 *p, int64_t i) {
    const uint64_t *q = reinterpret_cast<const uint64_t *>(p) + 2 * i;
    return u128{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
}
__device__ __forceinline__ void st(u128 *p, int64_t i, u128 v) {
    reinterpret_cast<ulonglong2 *>(p)[i] = make_ulonglong2(v.lo, v.hi);
}
// A store of streamed output that is not read again soon (non-temporal hint);
// one 16-byte store.
typedef unsigned long long ct_u64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(u128 *p, int64_t i, u128 v) {
    __builtin_nontemporal_store(ct_u64x2{v.lo, v.hi}, reinterpret_cast<ct_u64x2 *>(p) + i);
}

// Exact accumulation of many values into four 64-bit cells with atomics
// whose results are not waited for: cell j receives the j-th 32-bit limb of
// each value, so no cell can wrap before 2^32 additions, and from_limbs
// recombines sum_j cell_j 2^{32 j} mod 2^128.  (atomic_add128 below needs the
// returned old low limb to carry, which makes the adding thread wait.)
__device__ __forceinline__ void atomic_add_limbs(unsigned long long *cell, u128 v) {
    const unsigned long long l[4] = {v.lo & 0xffffffffull, v.lo >> 32, v.hi & 0xffffffffull, v.hi >> 32};
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (l[j]) atomicAdd(cell + j, l[j]);
}
__device__ __forceinline__ void from_limbs(const unsigned long long *cell, u128 &v) {
    const unsigned long long l0 = cell[0], l1 = cell[1], l2 = cell[2], l3 = cell[3];
    const unsigned long long lo = l0 + (l1 << 32);
    v = u128{lo, (l1 >> 32) + l2 + (l3 << 32) + (lo < l0 ? 1ull : 0ull)};
}

// Exact accumulation into a Z_{2^128} cell from many threads: the low limb is
// added atomically, and its wrap-around (old + v.lo >= 2^64) is carried into
// the high limb by a second atomic add.  Every wrap of the low word is counted
// exactly once, so the result is the mod-2^128 sum whatever the order.
__device__ __forceinline__ void atomic_add128(u128 *p, u128 v) {
    unsigned long long *q = reinterpret_cast<unsigned long long *>(p);
    const unsigned long long old = atomicAdd(q, (unsigned long long)v.lo);
    const unsigned long long carry = (old + v.lo < old) ? 1ull : 0ull;
    const unsigned long long hi = v.hi + carry;
    if (hi) atomicAdd(q + 1, hi);
}

// Orders a wavefront's LDS writes before its later LDS reads by other lanes
// of the same wavefront (a compiler and memory fence at wavefront scope).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// atomic_add128 of NV values into the cells p[i] with ok[i] set, the NV
// low-limb atomics in flight together before the first carry is formed (the
// empty asm keeps the compiler from merging each cell's two conditional
// blocks, which would wait for every atomic in turn).
template <int NV>
__device__ __forceinline__ void atomic_add128_n(u128 *const (&p)[NV], const u128 (&v)[NV], const bool (&ok)[NV]) {
    unsigned long long old[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) {
        old[i] = 0;
        if (ok[i]) old[i] = atomicAdd(reinterpret_cast<unsigned long long *>(p[i]), (unsigned long long)v[i].lo);
    }
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const unsigned long long hi = v[i].hi + (old[i] + v[i].lo < old[i] ? 1ull : 0ull);
        if (ok[i] && hi) atomicAdd(reinterpret_cast<unsigned long long *>(p[i]) + 1, hi);
    }
}

// atomic_add128 of v[i] into cell base[off[i] + at] for every i < NV, in
// flight together.
template <int NV, class R>
__device__ __forceinline__ void add_cells(R *base, const int64_t (&off)[NV], int64_t at, const R (&v)[NV]) {
    R *cell[NV];
    bool ok[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) {
        cell[i] = base + off[i] + at;
        ok[i] = true;
    }
    atomic_add128_n<NV>(cell, v, ok);
}

// ---------------------------------------------------------------- generator
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), counter form: the i-th draw of
// a stream with key `key` is mix(key + (i + 1) * golden gamma).

__device__ __forceinline__ uint64_t smix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sdraw(uint64_t key, uint64_t i) {
    return smix(key + (i + 1) * 0x9E3779B97F4A7C15ull);
}
__device__ __forceinline__ u128 sdraw128(uint64_t key, uint64_t e) {
    return u128{sdraw(key, 2 * e), sdraw(key, 2 * e + 1)};
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ u128 shfl_xor128(u128 v, int m) {
    u128 r;
    r.lo = __shfl_xor(v.lo, m, 64);
    r.hi = __shfl_xor(v.hi, m, 64);
    return r;
}
// sum over the 64 lanes of a wavefront (every lane receives the total)
__device__ __forceinline__ u128 wave_sum(u128 v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = add(v, shfl_xor128(v, m));
    return v;
}

// ---------------------------------------------------------------- Z_{2^64}
// The same operations for the k = s = 32 parameter set, whose shares and tags
// are elements of Z_{2^64}.

__device__ __forceinline__ r64 add(r64 a, r64 b) { return r64{a.v + b.v}; }
__device__ __forceinline__ r64 sub(r64 a, r64 b) { return r64{a.v - b.v}; }
__device__ __forceinline__ r64 mul(r64 a, r64 b) { return r64{a.v * b.v}; }
__device__ __forceinline__ r64 mul64(r64 a, uint64_t b) { return r64{a.v * b}; }
__device__ __forceinline__ r64 mad64(r64 acc, r64 a, uint64_t b) { return r64{acc.v + a.v * b}; }
__device__ __forceinline__ r64 mad(r64 acc, r64 a, r64 b) { return r64{acc.v + a.v * b.v}; }
__device__ __forceinline__ r64 ld(const r64 *p, int64_t i) { return p[i]; }
__device__ __forceinline__ r64 ld_nt(const r64 *p, int64_t i) { return r64{__builtin_nontemporal_load(&p[i].v)}; }
__device__ __forceinline__ void st(r64 *p, int64_t i, r64 v) { p[i] = v; }
__device__ __forceinline__ void st_nt(r64 *p, int64_t i, r64 v) { __builtin_nontemporal_store(v.v, &p[i].v); }
__device__ __forceinline__ void atomic_add_limbs(unsigned long long *cell, r64 v) {
    const unsigned long long l0 = v.v & 0xffffffffull, l1 = v.v >> 32;
    if (l0) atomicAdd(cell, l0);
    if (l1) atomicAdd(cell + 1, l1);
}
__device__ __forceinline__ void from_limbs(const unsigned long long *cell, r64 &v) { v = r64{cell[0] + (cell[1] << 32)}; }
__device__ __forceinline__ void atomic_add128(r64 *p, r64 v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v.v);
}
template <int NV>
__device__ __forceinline__ void atomic_add128_n(r64 *const (&p)[NV], const r64 (&v)[NV], const bool (&ok)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; i++)
        if (ok[i]) atomicAdd(reinterpret_cast<unsigned long long *>(p[i]), (unsigned long long)v[i].v);
}
__device__ __forceinline__ r64 shfl_xor128(r64 v, int m) { return r64{__shfl_xor(v.v, m, 64)}; }
__device__ __forceinline__ r64 wave_sum(r64 v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = add(v, shfl_xor128(v, m));
    return v;
}

// What depends on the parameter set, for element type R:
//   zero(), draw(key, e)  -- element e of a uniform stream of Z_{2^{k+s}}
//                            (for Z_{2^64}: the low half of the 128-bit element),
//   mod_s(x)              -- a draw as a key share or combiner in Z_{2^s},
//   mod_k(v)              -- the value v mod 2^k, as an integer,
//   lift(lo, up)          -- lo + 2^k up (lo < 2^k, up a draw),
//   input(draw, bits)     -- an input of Z_{2^k} (uniform, or signed bits-bit),
//   small(x)              -- an integer x < 2^64 as an element,
//   DIGITS                -- balanced base-256 digits per element.
template <class R>
struct Ring;

template <>
struct Ring<u128> {
    static constexpr int DIGITS = 16;
    __device__ static u128 zero() { return u128{0, 0}; }
    __device__ static u128 draw(uint64_t key, uint64_t e) { return sdraw128(key, e); }
    __device__ static uint64_t mod_s(uint64_t x) { return x; }
    __device__ static uint64_t mod_k(u128 v) { return v.lo; }
    __device__ static u128 lift(uint64_t lo, uint64_t up) { return u128{lo, up}; }
    __device__ static u128 input(uint64_t draw, int bits) {
        if (bits <= 0 || bits >= 64) return u128{draw, 0};
        return u128{(uint64_t)((int64_t)draw >> (64 - bits)), 0};
    }
    __device__ static u128 small(uint64_t x) { return u128{x, 0}; }
    __device__ static bool nonzero(u128 v) { return (v.lo | v.hi) != 0; }
    __device__ static ct_u128 out(u128 v) { return ct_u128{v.lo, v.hi}; }
};

template <>
struct Ring<r64> {
    static constexpr int DIGITS = 8;
    __device__ static r64 zero() { return r64{0}; }
    __device__ static r64 draw(uint64_t key, uint64_t e) { return r64{sdraw(key, 2 * e)}; }
    __device__ static uint64_t mod_s(uint64_t x) { return x & 0xFFFFFFFFull; }
    __device__ static uint64_t mod_k(r64 v) { return v.v & 0xFFFFFFFFull; }
    __device__ static r64 lift(uint64_t lo, uint64_t up) { return r64{lo | (up << 32)}; }
    __device__ static r64 input(uint64_t draw, int bits) {
        const uint32_t x = (uint32_t)draw;
        if (bits <= 0 || bits >= 32) return r64{x};
        return r64{(uint32_t)((int32_t)x >> (32 - bits))};
    }
    __device__ static r64 small(uint64_t x) { return r64{x}; }
    __device__ static bool nonzero(r64 v) { return v.v != 0; }
    __device__ static ct_u128 out(r64 v) { return ct_u128{v.v, 0}; }
};

// Sum of NV values over a block of WAVES wavefronts; the result is valid in
// thread 0.  `sh` must hold NV * WAVES entries.
template <int NV, int WAVES, class R>
__device__ __forceinline__ void block_sum(R (&v)[NV], R *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; i++) v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++) sh[i * WAVES + w] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++) {
            R s = sh[i * WAVES];
#pragma unroll
            for (int j = 1; j < WAVES; j++) s = add(s, sh[i * WAVES + j]);
            v[i] = s;
        }
    }
    __syncthreads();
}

}  // namespace ct
