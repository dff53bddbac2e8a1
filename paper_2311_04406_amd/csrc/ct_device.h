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
__device__ __forceinline__ void st(u128 *p, int64_t i, u128 v) {
    reinterpret_cast<ulonglong2 *>(p)[i] = make_ulonglong2(v.lo, v.hi);
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

// Sum of NV values over a block of WAVES wavefronts; the result is valid in
// thread 0.  `sh` must hold NV * WAVES entries.
template <int NV, int WAVES>
__device__ __forceinline__ void block_sum(u128 (&v)[NV], u128 *sh) {
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
            u128 s = sh[i * WAVES];
#pragma unroll
            for (int j = 1; j < WAVES; j++) s = add(s, sh[i * WAVES + j]);
            v[i] = s;
        }
    }
    __syncthreads();
}

}  // namespace ct
