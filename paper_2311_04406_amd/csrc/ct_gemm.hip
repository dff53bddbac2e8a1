// ct_gemm.hip -- exact matrix products over Z_{2^128} for gfx950.
//
// The local products of Eqs. (2)-(3) (E [B]_p, [A]_p U, E U and their tag
// counterparts) are dense contractions of 128-bit ring elements.  They run on
// the int8 matrix cores (v_mfma_i32_32x32x32_i8) through an exact digit
// decomposition:
//
//   x = sum_{d<16} x_d 2^{8d} (mod 2^128),  x_d in [-128, 127]  (balanced digits)
//   a*b mod 2^128 = sum_{t<16} 2^{8t} S_t,  S_t = sum_{i+j=t} a_i b_j
//
// so one 128-bit multiply-accumulate is 136 signed 8-bit digit products
// (pairs with i + j <= 15), grouped into 16 int32 "diagonal" accumulators.
// |a_i b_j| <= 2^14, so diagonal t over a K range of length L stays below
// (t + 1) * L * 2^14 <= 16 * L * 2^14 in magnitude; with L <= 255 * 32 every
// diagonal is exact in int32 and the host splits longer K ranges.  Partial
// results of K splits are combined with exact 128-bit atomic additions.
//
// Balanced digits of x are the bytes of (x + 0x8080...80) mod 2^128, each
// xored with 0x80 and read as int8: adding 128 to every digit of the balanced
// form gives a digit string in [0, 255], i.e. the ordinary bytes of x + K.
//
// Data flow.  k_pack converts every operand once into digit tiles (64 major
// indices x 32 k, 16 planes, 32 KB; layout in ct_internal.h) through an LDS
// transpose.  k_ring_gemm then only copies tiles: a workgroup of 4
// wavefronts owns a 64 x 64 output tile (32 x 32 per wavefront), streams one
// 32-wide K slice at a time (A and B tiles, 64 KB) global -> LDS with
// global_load_lds_dwordx4 into one of two statically distinct LDS stages
// while the matrix cores work on the other, and reads 16-byte digit fragments
// in a triangular order (fragment pair t unlocks 2t+1 or 2(16-t) products) so
// the first products issue after a single fragment pair.  k_ring_gemm_rs
// (the default) streams each wavefront's fragments straight into registers
// instead.  k_open_pack opens U and writes the right operands' tiles in one
// pass, and k_online_persist runs a whole two-party online phase as one
// persistent launch over the stage bodies.
#include "ct_passes.h"

namespace ct {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int PLANE = BM * BK;  // bytes per digit plane of a 64 x 32 tile

// Tile geometry per ring: NB digit planes per operand tile (OPB bytes, which
// is TILE_ELEMS elements).  A wavefront holds NB diagonal accumulators of 16
// registers per 32 x 32 output tile; with 8 digits (Z_{2^64}) that is half
// its 256 AGPRs, so it can take MT = 2 output tiles stacked in M (a workgroup
// then owns 64 MT x 64 outputs).  An LDS stage (Stage<R, MT>) holds the MT
// left-operand digit tiles and the right-operand digit tile of one K slice.
template <class R>
struct Tile {
    static constexpr int NB = Ring<R>::DIGITS;
    static constexpr int NW = NB / 4;            // 32-bit words of digits per element
    static constexpr int OPB = NB * PLANE;       // 32 KB (Z_{2^128}) or 16 KB (Z_{2^64})
    static constexpr int MT_MAX = NB == 8 ? 2 : 1;
    static_assert(OPB == TILE_ELEMS * (int)sizeof(R), "tile size");
};
template <class R, int MT>
constexpr int stage_bytes() { return (MT + 1) * Tile<R>::OPB; }

__device__ __forceinline__ void to_digits(r64 x, uint32_t (&w)[2]) {
    const uint64_t K = 0x8080808080808080ull;
    const uint64_t v = (x.v + K) ^ K;
    w[0] = (uint32_t)v;
    w[1] = (uint32_t)(v >> 32);
}

__device__ __forceinline__ void to_digits(u128 x, uint32_t (&w)[4]) {
    const uint64_t K = 0x8080808080808080ull;
    const uint64_t lo = x.lo + K;
    const uint64_t hi = x.hi + K + (lo < K ? 1ull : 0ull);
    w[0] = (uint32_t)(lo ^ K);
    w[1] = (uint32_t)((lo ^ K) >> 32);
    w[2] = (uint32_t)(hi ^ K);
    w[3] = (uint32_t)((hi ^ K) >> 32);
}

// byte offset of (major j, k) inside one digit plane (k a multiple of 8).
// Rows are 32 bytes; the two 16-byte halves of row j swap when bit 2 xor
// bit 3 of j is set, so the 16-byte fragment reads of 8 consecutive lanes
// (rows j..j+7) cover 32 distinct banks and those of 16 consecutive lanes
// cover 64.
__device__ __forceinline__ int half_swap(int j) { return ((j >> 2) ^ (j >> 3)) & 1; }
__device__ __forceinline__ int plane_off(int j, int k) {
    const int chunk = k >> 4;
    return j * BK + ((chunk ^ half_swap(j)) << 4) + (k & 15);
}

// Transposes the digits of 8 consecutive-k elements into 4 NW planes of 8
// bytes and writes them at base + d * PLANE + off.
template <int NW>
__device__ __forceinline__ void write_planes(uint8_t *base, int off, const uint32_t (&w)[8][NW]) {
#pragma unroll
    for (int q = 0; q < NW; q++) {  // dword q holds digits 4q .. 4q+3
        uint32_t y[2][4];
#pragma unroll
        for (int h = 0; h < 2; h++) {  // elements 4h .. 4h+3
            const uint32_t x0 = w[4 * h + 0][q], x1 = w[4 * h + 1][q];
            const uint32_t x2 = w[4 * h + 2][q], x3 = w[4 * h + 3][q];
            const uint32_t t0 = __builtin_amdgcn_perm(x1, x0, 0x05010400u);
            const uint32_t t1 = __builtin_amdgcn_perm(x1, x0, 0x07030602u);
            const uint32_t t2 = __builtin_amdgcn_perm(x3, x2, 0x05010400u);
            const uint32_t t3 = __builtin_amdgcn_perm(x3, x2, 0x07030602u);
            y[h][0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
            y[h][1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
            y[h][2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
            y[h][3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
        }
#pragma unroll
        for (int b = 0; b < 4; b++) {
            uint2 v = make_uint2(y[0][b], y[1][b]);
            *reinterpret_cast<uint2 *>(base + (4 * q + b) * PLANE + off) = v;
        }
    }
}

// ---------------------------------------------------------------- packing
// One workgroup per digit tile: 256 threads hold 8 consecutive-k elements
// each (a row segment of a left operand, staged through LDS; a column
// segment of a right one, loaded directly), write their digit planes to
// LDS, and the tile is stored with 16-byte coalesced writes.
template <class R>
__device__ __forceinline__ void pack_body(const PackJob *__restrict__ jobs, int njobs, int total_tiles, const Grid &g) {
    constexpr int OPBYTES = Tile<R>::OPB, NW = Tile<R>::NW;
    __shared__ __attribute__((aligned(16))) uint8_t tile[OPBYTES];
    const int tid = threadIdx.x;
    for (int t = (int)g.x; t < total_tiles; t += (int)g.nx) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        const PackJob J = jobs[lo];
        const int local = t - J.tile_begin;
        const int tm = local / J.kt, ks = local % J.kt;
        int j, kk;
        if (J.side == 0) { j = tid >> 2; kk = (tid & 3) * 8; }
        else { j = tid & 63; kk = (tid >> 6) * 8; }
        const int major = tm * 64 + j;
        const R *src = reinterpret_cast<const R *>(J.src);
        uint32_t w[8][NW];
        if (J.side == 0) {
            // a left operand's rows lie K elements apart: each load
            // instruction takes two whole 32-element row segments (lane =
            // element), the elements are staged in LDS with the 16 units of a
            // row half permuted by the row (so that both these writes and the
            // per-thread reads of 8 consecutive elements below spread over
            // the banks), and each thread reads back its 8.  (Loading the 8
            // directly took 16 bytes from each of 64 lines per instruction:
            // 1.8x the bytes from HBM and 27% more time on the batched set.)
            R *raw = reinterpret_cast<R *>(tile);
            const int lane = tid & 63, wv = tid >> 6;
            R e[8];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int r = 16 * wv + 2 * i + (lane >> 5), k = lane & 31;
                const int gm = tm * 64 + r, gk = ks * 32 + k;
                e[i] = gm < J.rows && gk < J.cols ? ld(src, (int64_t)gm * J.cols + gk) : Ring<R>::zero();
            }
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int r = 16 * wv + 2 * i + (lane >> 5), k = lane & 31;
                raw[r * 32 + (k ^ (r & 15))] = e[i];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 8; i++) to_digits(raw[j * 32 + ((kk + i) ^ (j & 15))], w[i]);
            __syncthreads();
        } else {
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int k = ks * 32 + kk + i;
                R v = Ring<R>::zero();
                if (k < J.rows && major < J.cols) {
                    // a convolution's right operand is the implicit im2col matrix of its input
                    const int64_t g = kn_src(J.cv, J.cols, k, major);
                    if (g >= 0) v = ld(src, g);
                }
                to_digits(v, w[i]);
            }
        }
        write_planes<NW>(tile, plane_off(j, kk), w);
        __syncthreads();
        uint4 *dst = reinterpret_cast<uint4 *>(reinterpret_cast<R *>(J.dst) + ((int64_t)tm * J.kt + ks) * TILE_ELEMS);
#pragma unroll
        for (int i = 0; i < OPBYTES / 16 / 256; i++)
            dst[i * 256 + tid] = reinterpret_cast<const uint4 *>(tile)[i * 256 + tid];
        __syncthreads();
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_pack(const PackJob *__restrict__ jobs, int njobs, int total_tiles) {
    pack_body<R>(jobs, njobs, total_tiles, hw_grid());
}

hipError_t launch_pack(int eb, const PackJob *jobs_dev, int njobs, int total_tiles, hipStream_t st) {
    if (njobs <= 0 || total_tiles <= 0) return hipSuccess;
    int grid = total_tiles < 65536 ? total_tiles : 65536;
    if (eb == 8) hipLaunchKernelGGL(k_pack<r64>, dim3(grid), dim3(256), 0, st, jobs_dev, njobs, total_tiles);
    else hipLaunchKernelGGL(k_pack<u128>, dim3(grid), dim3(256), 0, st, jobs_dev, njobs, total_tiles);
    return hipGetLastError();
}

// ---------------------------------------------------------------- open U and pack
// Two-party matrix-core layers that are not convolutions: one pass over
// K x N opens U = ([Y]_0 - [B]_0) + ([Y]_1 - [B]_1) (Fig. 7 online step 1),
// accumulates its batch check sums (Pi_BatchRec, Fig. 1), forms U^c and
// [tB^c]_p (compression along N, Pi_Compress) and writes the digit tiles of
// the right operands [B]_0, [B]_1 and U of the products -- the work of
// k_open_u and of k_pack's right-operand jobs, without reading [B]_p and U a
// second time.  One workgroup per 64 (n) x 32 (k) tile, laid out as k_pack
// lays out a right operand's tile: lane j takes column n = 64 tn + j,
// wavefront w the 8 rows k = 32 ks + 8 w + i; the rows' compressions are
// summed over the wavefront and added atomically, once per row and tile.
template <class R>
__device__ __forceinline__ void store_tile(uint8_t *tile, int off, const uint32_t (&w)[8][Tile<R>::NW], u128 *dst) {
    constexpr int OPB = Tile<R>::OPB;
    write_planes<Tile<R>::NW>(tile, off, w);
    __syncthreads();
    uint4 *d = reinterpret_cast<uint4 *>(dst);
#pragma unroll
    for (int i = 0; i < OPB / 16 / 256; i++) d[i * 256 + threadIdx.x] = reinterpret_cast<const uint4 *>(tile)[i * 256 + threadIdx.x];
    __syncthreads();
}

template <class R>
__device__ __forceinline__ void open_pack_body(const LayerDev *__restrict__ Ls, int flags, const Grid &g) {
    constexpr int NW = Tile<R>::NW;
    __shared__ __attribute__((aligned(16))) uint8_t tile[Tile<R>::OPB];
    __shared__ R sh[3 * WAVES];
    const LayerDev &L = Ls[g.y];
    if (!L.fo) return;
    const int64_t K = L.K, N = L.N;
    const int kt = (int)((K + 31) / 32), tiles = (int)((N + 63) / 64) * kt;
    if ((int)g.x >= tiles) return;
    const int tn = (int)g.x / kt, ks = (int)g.x - tn * kt;
    const int lane = threadIdx.x & 63, kk = (threadIdx.x >> 6) * 8;
    const int64_t n = (int64_t)tn * 64 + lane;
    const bool check = flags & F_CHECK, compact = (flags & F_COMPACT) && !L.cm;
    const bool need_tb = check || compact;
    const CvecOff o = cvec_off(L.M, K);
    const uint64_t kcu = L.key[K_CHI_U];
    const uint64_t xn = compact && n < N ? Ring<R>::mod_s(sdraw(L.key[K_CHI], (uint64_t)n)) : 0;
    R chk[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    uint32_t wb0[8][NW], wb1[8][NW], wu[8][NW];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int64_t k = (int64_t)ks * 32 + kk + i;
        R b0 = Ring<R>::zero(), b1 = Ring<R>::zero(), u = Ring<R>::zero();
        R tb0 = Ring<R>::zero(), tb1 = Ring<R>::zero();
        if (k < K && n < N) {
            const int64_t e = k * N + n;
            // all loads of the element before the store of U
            const R y0 = ld_nt(P<R>(L.Y[0]), e), y1 = ld_nt(P<R>(L.Y[1]), e);
            b0 = ld_nt(P<R>(L.B[0]), e);
            b1 = ld_nt(P<R>(L.B[1]), e);
            R ty0 = Ring<R>::zero(), ty1 = Ring<R>::zero();
            if (need_tb) {
                tb0 = ld_nt(P<R>(L.tB[0]), e);
                tb1 = ld_nt(P<R>(L.tB[1]), e);
            }
            if (check) {
                ty0 = ld_nt(P<R>(L.tY[0]), e);
                ty1 = ld_nt(P<R>(L.tY[1]), e);
            }
            u = add(sub(y0, b0), sub(y1, b1));
            // U is read again only by the column tags of a layer compressed along M
            if (L.cm) st(P<R>(L.U), e, u);
            else st_nt(P<R>(L.U), e, u);
            if (check) {
                const uint64_t x = Ring<R>::mod_s(sdraw(kcu, (uint64_t)e));
                chk[0] = mad64(chk[0], sub(ty0, tb0), x);
                chk[1] = mad64(chk[1], sub(ty1, tb1), x);
                chk[2] = mad64(chk[2], u, x);
            }
        }
        if (compact && k < K) {  // k is the same for the whole wavefront
            const R v0 = wave_sum(mul64(u, xn)), v1 = wave_sum(mul64(tb0, xn)), v2 = wave_sum(mul64(tb1, xn));
            if (lane == 0) add_cells<3>(P<R>(L.cvec), {o.Uc, o.tBc0, o.tBc1}, k, {v0, v1, v2});
        }
        to_digits(b0, wb0[i]);
        to_digits(b1, wb1[i]);
        to_digits(u, wu[i]);
    }
    const int64_t toff = ((int64_t)tn * kt + ks) * TILE_ELEMS;
    const int off = plane_off(lane, kk);
    store_tile<R>(tile, off, wb0, reinterpret_cast<u128 *>(P<R>(L.rp[0]) + toff));
    store_tile<R>(tile, off, wb1, reinterpret_cast<u128 *>(P<R>(L.rp[1]) + toff));
    store_tile<R>(tile, off, wu, reinterpret_cast<u128 *>(P<R>(L.rp[2]) + toff));
    if (check) block_accumulate<3>(chk, sh, P<R>(L.acc) + 3);
}

template <class R>
__global__ __launch_bounds__(256) void k_open_pack(const LayerDev *__restrict__ Ls, int flags) {
    open_pack_body<R>(Ls, flags, hw_grid());
}

hipError_t launch_open_pack(int eb, const LayerDev *L, int n, int flags, int max_tiles, hipStream_t st) {
    if (n <= 0 || max_tiles <= 0) return hipSuccess;
    LAUNCH_RING(eb, k_open_pack, dim3(max_tiles, n), dim3(256), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- products

// 2^sh * s (s a signed 32-bit diagonal sum) as an element of Z_{2^128}
template <int SH>
__device__ __forceinline__ u128 shifted(int32_t s) {
    const int64_t x = (int64_t)s;
    if constexpr (SH == 0) {
        return u128{(uint64_t)x, (uint64_t)(x >> 63)};
    } else if constexpr (SH < 64) {
        return u128{(uint64_t)x << SH, (uint64_t)(x >> (64 - SH))};
    } else {
        return u128{0, (uint64_t)x << (SH - 64)};
    }
}

template <int T>
__device__ __forceinline__ void combine(const v16i (&acc)[16], int r, u128 &v) {
    if constexpr (T < 16) {
        v = add(v, shifted<8 * T>(acc[T][r]));
        combine<T + 1>(acc, r, v);
    }
}
// Z_{2^64}: sum_{t<8} 2^{8t} S_t mod 2^64
template <int T>
__device__ __forceinline__ void combine(const v16i (&acc)[8], int r, r64 &v) {
    if constexpr (T < 8) {
        v.v += (uint64_t)(int64_t)acc[T][r] << (8 * T);
        combine<T + 1>(acc, r, v);
    }
}

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ const uint8_t *uniform_ptr(const uint8_t *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const uint8_t *>(((uint64_t)hi << 32) | lo);
}

// Copies the MT left and the right digit tiles of one K slice into an LDS
// stage (left tiles first): chunks of 1 KB, (MT + 1) OPB / 4 KB per
// wavefront, each a single global_load_lds_dwordx4 (lane l moves bytes
// [16 l, 16 l + 16) of its chunk).  Every chunk's tile base is made
// wavefront-uniform so each copy addresses memory as scalar base + 32-bit
// lane offset (no 64-bit address registers to keep live across the
// products).  A left tile past the operand's last row tile (null) is not
// copied: its rows are not stored.
template <class R, int MT>
__device__ __forceinline__ void issue_slice(const uint8_t *const (&a_tiles)[MT], const uint8_t *b_tile,
                                            uint8_t *stage) {
    constexpr int TCH = Tile<R>::OPB / 1024;  // chunks per tile
    constexpr int CH = (MT + 1) * TCH / 4;                       // chunks per wavefront
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int i = 0; i < CH; i++) {
        const int c = wave * CH + i, q = c / TCH;
        const uint8_t *src = q < MT ? a_tiles[q < MT ? q : 0] : b_tile;
        if (!src) continue;
        const uint8_t *base = uniform_ptr(src);
        __builtin_amdgcn_global_load_lds((const void *)(base + (uint32_t)(c - q * TCH) * 1024 + lane * 16),
                                         (lds_void *)(stage + c * 1024), 16, 0, 0);
    }
}

// Digit plane t of a fragment whose plane-0 byte offset in an LDS stage is off.
__device__ __forceinline__ v4i frag(const uint8_t *stage, int off, int t) {
    return *reinterpret_cast<const v4i *>(stage + off + t * PLANE);
}

// Product group T of a K slice: the digit pairs (T, j), j <= T, and (i, T),
// i < T, with digit sum below NB -- the products that fragment pair T
// completes -- for each of the MT output tiles (which share the right
// fragments).  Group sizes 1, 3, 5, ... up to NB / 2, then 2 (NB - T), times MT.
template <int NB, int MT>
__device__ __forceinline__ void group_products(int T, const v4i (&a)[MT][NB], const v4i (&b)[NB],
                                               v16i (&acc)[MT][NB]) {
#pragma unroll
    for (int j = 0; j < NB; j++)
#pragma unroll
        for (int h = 0; h < MT; h++)
            if (j <= T && T + j < NB)
                acc[h][T + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[h][T], b[j], acc[h][T + j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
        for (int h = 0; h < MT; h++)
            if (i < T && i + T < NB)
                acc[h][i + T] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[h][i], b[T], acc[h][i + T], 0, 0, 0);
}

// Adds v into out[idx] exactly mod 2^{k+s} for the outputs with ok set, all
// 16 atomics of a lane in flight together (an output out of range issues
// nothing).
template <class R>
__device__ __forceinline__ void add_outputs(R *out, const int64_t (&idx)[16], const bool (&ok)[16], const R (&v)[16]) {
    R *cell[16];
#pragma unroll
    for (int r = 0; r < 16; r++) cell[r] = out + idx[r];
    atomic_add128_n<16>(cell, v, ok);
}

// Epilogue of a wavefront's MT output tiles: the 32x32 accumulator layout
// gives lane l, register r row 8*(r/4) + 4*(l/32) + r%4 and column l%32 of
// an output tile; each output is sum_t 2^{8t} S_t plus the base (or added
// atomically to the output when the product's K range is split).  A lane's
// 16 outputs of a tile are formed first and their base loads (or atomics)
// issued together, so the wavefront waits for memory once per tile rather
// than once per output.  Both streams are non-temporal: read and written
// once here, they would only displace operand tiles from L2.
template <class R, int MT>
__device__ __forceinline__ void store_tile_out(const GemmProb &P, const v16i (&acc)[MT][Tile<R>::NB], int m0, int n0,
                                               int wm, int wn, int lane) {
    const int M = P.M, N = P.N;
    const int col = n0 + wn * 32 + (lane & 31);
    R *out = reinterpret_cast<R *>(P.out);
    const R *base = reinterpret_cast<const R *>(P.base);
#pragma unroll
    for (int h = 0; h < MT; h++) {
        const int row0 = m0 + 32 * (MT * wm + h) + 4 * (lane >> 5);
        R v[16];
        int64_t idx[16];
        bool ok[16];
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int row = row0 + 8 * (r >> 2) + (r & 3);
            ok[r] = row < M && col < N;
            idx[r] = (int64_t)row * N + col;
            v[r] = Ring<R>::zero();
            combine<0>(acc[h], r, v[r]);
        }
        if (P.accumulate) {
            add_outputs(out, idx, ok, v);
        } else {
            if (base) {
                R b[16];
#pragma unroll
                for (int r = 0; r < 16; r++) b[r] = ok[r] ? ld_nt(base, idx[r]) : Ring<R>::zero();
#pragma unroll
                for (int r = 0; r < 16; r++) v[r] = add(v[r], b[r]);
            }
#pragma unroll
            for (int r = 0; r < 16; r++)
                if (ok[r]) st_nt(out, idx[r], v[r]);
        }
    }
}

// vmcnt(0), expcnt and lgkmcnt left unconstrained (gfx9 s_waitcnt encoding)
#define WAIT_VMEM() __builtin_amdgcn_s_waitcnt(0x0F70)

template <class R, int MT>
__device__ __forceinline__ void gemm_tile(const GemmProb &P, int tm, int tn, int split, uint8_t *lds) {
    constexpr int NB = Tile<R>::NB, OPB = Tile<R>::OPB, STAGE = stage_bytes<R, MT>();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = P.M;
    const int m0 = tm * 64 * MT, n0 = tn * BN;
    const int s_begin = split * P.steps_per_split;
    const int s_end = min(s_begin + P.steps_per_split, P.nsteps);
    const int mtiles = (M + 63) / 64;  // row tiles of the packed left operand

    v16i acc[MT][NB];
#pragma unroll
    for (int h = 0; h < MT; h++)
#pragma unroll
        for (int t = 0; t < NB; t++) acc[h][t] = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

    auto copy_slice = [&](int step, uint8_t *stage) {
        const int seg = step >= P.kt ? 1 : 0, ks = step - seg * P.kt;
        const R *Lp = reinterpret_cast<const R *>(seg ? P.Lp2 : P.Lp1);
        const R *Rp = reinterpret_cast<const R *>(seg ? P.Rp2 : P.Rp1);
        const uint8_t *at[MT];
#pragma unroll
        for (int q = 0; q < MT; q++) {
            const int t = tm * MT + q;
            at[q] = t < mtiles ? reinterpret_cast<const uint8_t *>(Lp + ((int64_t)t * P.kt + ks) * TILE_ELEMS) : nullptr;
        }
        issue_slice<R, MT>(at, reinterpret_cast<const uint8_t *>(Rp + ((int64_t)tn * P.kt + ks) * TILE_ELEMS), stage);
    };

    // MFMA-side fragment offsets: lane -> row/column lane % 32, k half lane / 32.
    // Output tile h of the wavefront has rows 32 (MT wm + h) + lane % 32 of the
    // workgroup's 64 MT, i.e. rows of left tile (MT wm + h) / 2.
    const int chunk = lane >> 5;
    int a_off[MT];
#pragma unroll
    for (int h = 0; h < MT; h++) {
        const int r = 32 * (MT * wm + h) + (lane & 31), q = r >> 6, lr = r & 63;
        a_off[h] = q * OPB + lr * BK + ((chunk ^ half_swap(lr)) << 4);
    }
    const int brow = wn * 32 + (lane & 31);
    const int b_off = MT * OPB + brow * BK + ((chunk ^ half_swap(brow)) << 4);

    // Software pipeline over K slices (LDS stages alternate):
    //   top of slice s: copy slice s+1 global -> LDS (the other stage);
    //   product group t reads fragment pair t+2 (two groups of products
    //   cover the LDS latency);
    //   after group NB-3 every fragment of slice s is in registers: wait for
    //   this wavefront's copies, barrier (slice s+1 has landed and no
    //   wavefront reads stage s any more), read fragment pairs 0 and 1 of
    //   slice s+1, then the last two groups of slice s hide their latency.
    // Scheduling barriers keep the compiler from regrouping the reads.
    v4i a[MT][NB], b[NB], a0n[MT], a1n[MT], b0n, b1n;
    if (s_begin < s_end) copy_slice(s_begin, lds);
    WAIT_VMEM();
    __syncthreads();
#pragma unroll
    for (int h = 0; h < MT; h++) {
        a[h][0] = frag(lds, a_off[h], 0);
        a[h][1] = frag(lds, a_off[h], 1);
    }
    b[0] = frag(lds, b_off, 0);
    b[1] = frag(lds, b_off, 1);
    for (int s = s_begin; s < s_end; s++) {
        const int buf = (s - s_begin) & 1;
        const uint8_t *stage = lds + buf * STAGE;
        uint8_t *next = lds + (buf ^ 1) * STAGE;
        const bool more = s + 1 < s_end;
        if (more) copy_slice(s + 1, next);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < NB; t++) {
            if (t + 2 < NB) {
#pragma unroll
                for (int h = 0; h < MT; h++) a[h][t + 2] = frag(stage, a_off[h], t + 2);
                b[t + 2] = frag(stage, b_off, t + 2);
            }
            group_products<NB, MT>(t, a, b, acc);
            __builtin_amdgcn_sched_barrier(0);
            if (t == NB - 3) {
                WAIT_VMEM();
                __syncthreads();
                if (more) {
#pragma unroll
                    for (int h = 0; h < MT; h++) {
                        a0n[h] = frag(next, a_off[h], 0);
                        a1n[h] = frag(next, a_off[h], 1);
                    }
                    b0n = frag(next, b_off, 0);
                    b1n = frag(next, b_off, 1);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int h = 0; h < MT; h++) {
            a[h][0] = a0n[h];
            a[h][1] = a1n[h];
        }
        b[0] = b0n;
        b[1] = b1n;
    }

    store_tile_out<R, MT>(P, acc, m0, n0, wm, wn, lane);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): block b runs on XCD b % 8.  With xcd_remap the tile list is cut into
// 8 contiguous ranges, one per XCD, so the workgroups resident on an XCD at a
// time work on neighbouring tiles.  The tiles of a layer's products (both
// parties; four products in SPDZ2k mode) are numbered together, from slowest
// to fastest: K split, group of group_m output row tiles, output column tile,
// product, row tile within the group.  Neighbouring tiles therefore read the
// same right-operand tile (all row tiles and both parties' products use U)
// and the same left-operand tiles (E is shared by all products) in the same
// K slice at about the same time.
// xcd_remap = 1: XCD x takes the x-th of 8 contiguous ranges of the list.
// xcd_remap = G >= 2: the list is cut into groups of G consecutive tiles and
// group g goes to XCD g % 8, whose blocks take their groups in order -- the
// G tiles of a group (e.g. the row tiles and products that share one right-
// operand tile) run on one XCD at about the same time and share its L2, and
// every XCD still works across the whole list.  The tail that does not fill
// 8 groups keeps the identity order.  Both are bijections on [0, total).
__device__ __forceinline__ int xcd_tile(int b, int total, int mode) {
    const int x = b & 7, i = b >> 3;
    if (mode == 1) {
        const int q = total >> 3, r = total & 7;
        return x * q + (x < r ? x : r) + i;
    }
    const int full = total / (8 * mode) * (8 * mode);
    if (b >= full) return b;
    return ((i / mode) * 8 + x) * mode + i % mode;
}

// Tile t of a launch -> (problem, output row tile, column tile, K split),
// in the order described above.
struct TileRef {
    int prob, tm, tn, split;
};
__device__ __forceinline__ TileRef decode_tile(const GemmProb *__restrict__ probs, int nprobs, int t) {
    int lo = 0, hi = nprobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const GemmProb &G = probs[lo];
    const int tiles_m = G.tiles_m, tiles_n = G.tiles_n, gsize = G.gsize, gm = G.group_m;
    const int local = t - G.tile_begin;
    const int per_split = tiles_m * tiles_n * gsize;
    const int split = local / per_split;
    const int rem = local - split * per_split;
    const int tmg = rem / (gm * tiles_n * gsize);
    const int gme = min(gm, tiles_m - tmg * gm);
    const int r2 = rem - tmg * gm * tiles_n * gsize;
    const int tn = r2 / (gme * gsize);
    const int r3 = r2 - tn * gme * gsize;
    const int pidx = r3 / gme;
    return TileRef{G.gfirst + pidx, tmg * gm + (r3 - pidx * gme), tn, split};
}

template <class R, int MT>
__global__ __launch_bounds__(256, 1) void k_ring_gemm(const GemmProb *__restrict__ probs, int nprobs,
                                                      int total_tiles, int xcd_remap) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[2 * stage_bytes<R, MT>()];
    for (int b = blockIdx.x; b < total_tiles; b += gridDim.x) {
        const int t = xcd_remap ? xcd_tile(b, total_tiles, xcd_remap) : b;
        const TileRef tr = decode_tile(probs, nprobs, t);
        const GemmProb P = probs[tr.prob];
        gemm_tile<R, MT>(P, tr.tm, tr.tn, tr.split, lds);
    }
}

// ---------------------------------------------------------------- products, register-streamed
// The same products without LDS: every wavefront loads its own digit
// fragments straight from the packed tiles in global memory into registers
// (16 bytes per lane, 1 KB per fragment and wavefront, coalesced), half a
// K slice ahead: before product group T of a slice runs, fragment pair
// T + RS_PREFETCH is loaded (of this slice, or of the next once past its
// end), so each load has half a slice of products to land and the wavefront
// never waits at a barrier (a whole slice ahead kept more registers live
// and measured 2-4% slower).  The two wavefronts of a
// workgroup that share a row (or column) tile read the same fragment at about
// the same time, so the second read is served by the compute unit's cache.
// Registers: the NB diagonal accumulators of MT output tiles in AGPRs; the
// current and the next slice's fragments in VGPRs (live ranges overlap by
// about half a slice in the triangular order).

// A digit tile of one K slice as a buffer resource: wavefront-uniform base
// (scalar registers), OPB bytes; a fragment load adds the lane's 32-bit
// offset and the plane's scalar offset, and anything past the tile would
// read as zero instead of leaving it.
typedef __amdgpu_buffer_rsrc_t tile_rsrc;
#ifndef RS_PREFETCH
#define RS_PREFETCH 8
#endif
constexpr int RSRC_FLAGS = 0x00020000;  // gfx9 buffer resource word 3: 32-bit data format

template <class R>
__device__ __forceinline__ tile_rsrc tile_buffer(const uint8_t *tile) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(tile), 0, Tile<R>::OPB, RSRC_FLAGS);
}

__device__ __forceinline__ v4i load_frag(tile_rsrc t, int lane_off, int plane_off) {
    return __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(t, lane_off, plane_off, 0));
}

// Loads fragment pair T (MT left fragments, one right fragment) of a slice.
template <class R, int MT>
__device__ __forceinline__ void load_pair(int T, const tile_rsrc (&at)[MT], tile_rsrc bt, const int (&a_off)[MT],
                                          int b_off, v4i (&a)[MT][Tile<R>::NB], v4i (&b)[Tile<R>::NB]) {
#pragma unroll
    for (int h = 0; h < MT; h++) a[h][T] = load_frag(at[h], a_off[h], T * PLANE);
    b[T] = load_frag(bt, b_off, T * PLANE);
}

// One K slice with a prefetch distance of D <= NB product groups: before group T
// the wavefront loads fragment pair T + D -- of this slice (tiles ct, cbt,
// into ca, cb) while T + D < NB, else pair T + D - NB of the next slice
// (tiles na, nbt, into xa, xb).  Pairs 0 .. D - 1 of a slice are therefore
// loaded during the previous one.
template <class R, int MT, int D>
__device__ __forceinline__ void rs_slice(v4i (&ca)[MT][Tile<R>::NB], v4i (&cb)[Tile<R>::NB],
                                         v4i (&xa)[MT][Tile<R>::NB], v4i (&xb)[Tile<R>::NB],
                                         const tile_rsrc (&ct)[MT], tile_rsrc cbt, const tile_rsrc (&na)[MT],
                                         tile_rsrc nbt, const int (&a_off)[MT], int b_off,
                                         v16i (&acc)[MT][Tile<R>::NB]) {
    constexpr int NB = Tile<R>::NB;
    static_assert(D >= 1 && D <= NB, "prefetch distance");
#pragma unroll
    for (int T = 0; T < NB; T++) {
        if (T + D < NB) load_pair<R, MT>(T + D, ct, cbt, a_off, b_off, ca, cb);
        else load_pair<R, MT>(T + D - NB, na, nbt, a_off, b_off, xa, xb);
        group_products<NB, MT>(T, ca, cb, acc);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <class R, int MT>
__device__ __forceinline__ void gemm_tile_rs(const GemmProb &P, int tm, int tn, int split) {
    constexpr int NB = Tile<R>::NB, OPB = Tile<R>::OPB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s_begin = split * P.steps_per_split;
    const int s_end = min(s_begin + P.steps_per_split, P.nsteps);
    const int mtiles = (P.M + 63) / 64;  // row tiles of the packed left operand

    // The wavefront's place in the workgroup tile (WaveShape; MT stacked
    // tiles only as 2 x 2) and its first output row r0 and column c0.  A
    // wavefront whose outputs all lie past M or N has nothing to store and
    // leaves (this kernel has no barriers).
    int r0, c0;
    if (MT == 1 && P.wshape == WS_32x128) {
        r0 = tm * 32;
        c0 = tn * 128 + 32 * wave;
    } else if (MT == 1 && P.wshape == WS_128x32) {
        r0 = tm * 128 + 32 * wave;
        c0 = tn * 32;
    } else {
        r0 = tm * 64 * MT + 32 * MT * (wave >> 1);
        c0 = tn * 64 + 32 * (wave & 1);
    }
    if (r0 >= P.M || c0 >= P.N) return;

    v16i acc[MT][NB];
#pragma unroll
    for (int h = 0; h < MT; h++)
#pragma unroll
        for (int t = 0; t < NB; t++) acc[h][t] = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

    // Lane -> row (column) lane % 32 of the wavefront's 32, 16-byte k half
    // lane / 32 (rows swap their halves as k_pack lays them out).  Output
    // tile h has rows r0 + 32 h + lane % 32, i.e. rows of packed left tile
    // a_q[h]; a missing last left tile (M past its rows) is read from the
    // first one, whose products are then not stored.  Columns c0 + lane % 32
    // lie in packed right tile c0 / 64.
    const int chunk = lane >> 5;
    int a_off[MT], a_q[MT];
#pragma unroll
    for (int h = 0; h < MT; h++) {
        const int r = r0 + 32 * h, lr = (r & 63) + (lane & 31);
        a_q[h] = (r >> 6) < mtiles ? (r >> 6) : 0;
        a_off[h] = lr * BK + ((chunk ^ half_swap(lr)) << 4);
    }
    const int b_q = c0 >> 6, lc = (c0 & 63) + (lane & 31);
    const int b_off = lc * BK + ((chunk ^ half_swap(lc)) << 4);

    // digit tiles of step st (a K slice of the first or second segment)
    auto tiles = [&](int st, tile_rsrc (&at)[MT], tile_rsrc &bt) {
        const int seg = st >= P.kt ? 1 : 0, ks = st - seg * P.kt;
        const uint8_t *Lp = reinterpret_cast<const uint8_t *>(seg ? P.Lp2 : P.Lp1);
        const uint8_t *Rp = reinterpret_cast<const uint8_t *>(seg ? P.Rp2 : P.Rp1);
#pragma unroll
        for (int h = 0; h < MT; h++)
            at[h] = tile_buffer<R>(uniform_ptr(Lp + ((int64_t)a_q[h] * P.kt + ks) * OPB));
        bt = tile_buffer<R>(uniform_ptr(Rp + ((int64_t)b_q * P.kt + ks) * OPB));
    };

    // fragments of two consecutive slices: fa[c], fb[c] hold slice s while
    // the first pairs of slice s + 1 arrive in fa[1 - c], fb[1 - c] (c
    // alternates; both indices are compile-time constants)
    constexpr int D = RS_PREFETCH < NB ? RS_PREFETCH : NB;  // at most a whole slice ahead
    v4i fa[2][MT][NB], fb[2][NB];
    tile_rsrc t0[MT], b0t, t1[MT], b1t;
    if (s_begin < s_end) {
        tiles(s_begin, t0, b0t);
#pragma unroll
        for (int T = 0; T < D; T++) load_pair<R, MT>(T, t0, b0t, a_off, b_off, fa[0], fb[0]);
    }
    // slices in pairs (the fragment sets alternate), then an odd last one;
    // the last slice of the range loads the first pairs of its own tiles
    // again (unused), so that no load is conditional
    const int nsl = s_end - s_begin;
    for (int s = s_begin; s + 1 < s_end; s += 2) {
        tiles(s + 1, t1, b1t);
        rs_slice<R, MT, D>(fa[0], fb[0], fa[1], fb[1], t0, b0t, t1, b1t, a_off, b_off, acc);
        tiles(min(s + 2, s_end - 1), t0, b0t);
        rs_slice<R, MT, D>(fa[1], fb[1], fa[0], fb[0], t1, b1t, t0, b0t, a_off, b_off, acc);
    }
    if (nsl > 0 && (nsl & 1))
        rs_slice<R, MT, D>(fa[0], fb[0], fa[1], fb[1], t0, b0t, t0, b0t, a_off, b_off, acc);
    store_tile_out<R, MT>(P, acc, r0, c0, 0, 0, lane);
}

// One workgroup per output tile (grid = total_tiles): a loop over tiles
// around the K loop would make the compiler wait for every outstanding load
// at the top of each K iteration (the epilogue's stores meet the prefetched
// loads at the loop header), which the prefetch is there to avoid.
template <class R, int MT>
__global__ __launch_bounds__(256, 1) void k_ring_gemm_rs(const GemmProb *__restrict__ probs, int nprobs,
                                                         int total_tiles, int xcd_remap) {
    const int b = blockIdx.x;
    if (b >= total_tiles) return;
    const int t = xcd_remap ? xcd_tile(b, total_tiles, xcd_remap) : b;
    const TileRef tr = decode_tile(probs, nprobs, t);
    const GemmProb P = probs[tr.prob];
    gemm_tile_rs<R, MT>(P, tr.tm, tr.tn, tr.split);
}

// ---------------------------------------------------------------- persistent launch
// The two-party online phase of a batch of matrix-core layers in one launch:
// one workgroup per compute unit walks the stages of the staged kernels, in
// their order, over every layer of the batch -- zeroing; opening U with the
// right operands' digit tiles; the pass over M x K; packing the left
// operands (and the constant terms of split products); the products; the
// pass over M x N; the compact tag's final step; the check verdicts -- as
// workgroups of grids of its own, running the same stage bodies.  A stage
// starts when every workgroup has finished the previous one (grid barrier).
// The register-streamed products need all 512 registers of a lane, so every
// stage runs at one workgroup (four wavefronts) per compute unit.

// Grid barrier: workgroup arrivals counted in sync[0] (phase p is complete
// at p * gridDim.x arrivals).  The release fence before the arrival and the
// acquire fence after the wait make the workgroups' writes of the earlier
// stages visible to the later ones on every XCD.  The wait is bounded: past
// `ticks` of the 100 MHz wall clock (2 s by default) it sets sync[1] and goes
// on, and a workgroup that sees sync[1] set stops waiting at once.
__device__ __forceinline__ void grid_barrier(uint32_t *sync, uint32_t phase, uint64_t ticks) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(sync, 1u);
        const uint32_t target = phase * gridDim.x;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(sync, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (wall_clock64() - t0 > ticks) {
                atomicOr(sync + 1, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        __threadfence();
    }
    __syncthreads();
}

template <class R, int MT>
__global__ __launch_bounds__(256, 1) void k_online_persist(PersistArgs a) {
    const uint32_t W = gridDim.x, w = blockIdx.x;
    uint32_t phase = 0;
    if (a.zero_what)
        for (int l = 0; l < a.n; l++) zero_acc_body<R>(a.Ls, a.zero_what, Grid{w, (uint32_t)l, W});
    grid_barrier(a.sync, ++phase, a.wait_ticks);
    // the right operands' tiles of all layers as one list, dealt round-robin
    uint32_t first = 0;
    for (int l = 0; l < a.n; l++) {
        const LayerDev &L = a.Ls[l];
        const uint32_t tiles = L.fo ? (uint32_t)(((L.N + 63) / 64) * ((L.K + 31) / 32)) : 0;
        for (uint32_t t = (w + W - first % W) % W; t < tiles; t += W) open_pack_body<R>(a.Ls, a.flags, Grid{t, (uint32_t)l, tiles});
        first += tiles;
    }
    grid_barrier(a.sync, ++phase, a.wait_ticks);  // the row pass reads U^c and [tB^c]_p
    for (int l = 0; l < a.n; l++) row_pass_layer<R, 0>(a.Ls, a.flags, Grid{w, (uint32_t)l, W});
    grid_barrier(a.sync, ++phase, a.wait_ticks);
    pack_body<R>(a.jobs, a.njobs, a.pack_tiles, Grid{w, 0, W});
    if (a.any_accum)
        for (int p = 0; p < a.nprobs; p++) prob_base_body<R>(a.probs, Grid{w, (uint32_t)p, W});
    grid_barrier(a.sync, ++phase, a.wait_ticks);
    // the product tiles are taken in list order as workgroups free up (tiles
    // differ in length), from one counter per XCD so that tile b still runs on
    // XCD b % 8 as in the staged kernel: counter x hands out b = 8 i + x (one
    // counter for all if the grid has fewer than 8 workgroups)
    {
        __shared__ int next_tile;
        const uint32_t q = W >= 8 ? 8 : 1, x = w % q;
        for (;;) {
            if (threadIdx.x == 0) next_tile = (int)(q * atomicAdd(a.sync + 4 + x, 1u) + x);
            __syncthreads();
            const int b = next_tile;
            __syncthreads();
            if (b >= a.total_tiles) break;
            const int t = a.xcd_remap ? xcd_tile(b, a.total_tiles, a.xcd_remap) : b;
            const TileRef tr = decode_tile(a.probs, a.nprobs, t);
            const GemmProb P = a.probs[tr.prob];
            gemm_tile_rs<R, MT>(P, tr.tm, tr.tn, tr.split);
        }
    }
    grid_barrier(a.sync, ++phase, a.wait_ticks);
    for (int l = 0; l < a.n; l++) post_body<R>(a.Ls, a.flags, Grid{w, (uint32_t)l, W});
    grid_barrier(a.sync, ++phase, a.wait_ticks);
    // four workgroups per layer, as the staged kernel
    if (a.flags & F_COMPACT)
        for (uint32_t v = w; v < 4u * (uint32_t)a.n; v += W) compact_final_body<R>(a.Ls, a.flags, Grid{v & 3, v >> 2, 4});
    grid_barrier(a.sync, ++phase, a.wait_ticks);
    // one wavefront per layer; a run-out barrier rejects every layer
    const bool ran_out = __hip_atomic_load(a.sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const int lane = threadIdx.x & 63;
    for (int l = (int)(w * WAVES + (threadIdx.x >> 6)); l < a.n; l += (int)(W * WAVES)) {
        finalize_body<R>(a.Ls, a.n, a.out, l);
        if (ran_out && lane == 0) {
            ct_check_result *r = a.out + a.Ls[l].out_index;
            r->accept = 0;
            r->reserved = 1;
        }
    }
}

hipError_t launch_online_persist(int eb, const PersistArgs &a, int wgs, hipStream_t st) {
    if (a.n <= 0 || wgs <= 0) return hipSuccess;
    if (eb == 8 && a.mt == 2)
        hipLaunchKernelGGL((k_online_persist<r64, 2>), dim3(wgs), dim3(256), 0, st, a);
    else if (eb == 8)
        hipLaunchKernelGGL((k_online_persist<r64, 1>), dim3(wgs), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_online_persist<u128, 1>), dim3(wgs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gemm(int eb, const GemmProb *probs_dev, int nprobs, int total_tiles, int xcd_remap, int mt,
                       int kernel, hipStream_t st) {
    if (nprobs <= 0 || total_tiles <= 0) return hipSuccess;
    if (kernel == GEMM_REGS) {
        if (eb == 8 && mt == 2)
            hipLaunchKernelGGL((k_ring_gemm_rs<r64, 2>), dim3(total_tiles), dim3(256), 0, st, probs_dev, nprobs,
                               total_tiles, xcd_remap);
        else if (eb == 8)
            hipLaunchKernelGGL((k_ring_gemm_rs<r64, 1>), dim3(total_tiles), dim3(256), 0, st, probs_dev, nprobs,
                               total_tiles, xcd_remap);
        else
            hipLaunchKernelGGL((k_ring_gemm_rs<u128, 1>), dim3(total_tiles), dim3(256), 0, st, probs_dev, nprobs,
                               total_tiles, xcd_remap);
        return hipGetLastError();
    }
    if (eb == 8 && mt == 2)
        hipLaunchKernelGGL((k_ring_gemm<r64, 2>), dim3(total_tiles), dim3(256), 0, st, probs_dev, nprobs, total_tiles,
                           xcd_remap);
    else if (eb == 8)
        hipLaunchKernelGGL((k_ring_gemm<r64, 1>), dim3(total_tiles), dim3(256), 0, st, probs_dev, nprobs, total_tiles,
                           xcd_remap);
    else
        hipLaunchKernelGGL((k_ring_gemm<u128, 1>), dim3(total_tiles), dim3(256), 0, st, probs_dev, nprobs,
                           total_tiles, xcd_remap);
    return hipGetLastError();
}

// ---------------------------------------------------------------- skinny
// The dealer's triple product C~ = A~ B~ for layers with few output columns
// (N <= SKINNY_MAX_N, e.g. a classifier layer at batch 1) is a bandwidth-bound
// row-times-matrix product: one wavefront per output row, lanes striding over
// K with coalesced 16-byte loads, 128-bit VALU multiply-adds, a wavefront
// reduction per column.  (The online phase forms these products inside its
// pass over E.)
template <class R>
__global__ __launch_bounds__(256) void k_skinny(const SkinnyProb *__restrict__ probs, int nprobs) {
    const SkinnyProb P = probs[blockIdx.y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int N = P.N, K = P.K;
    const R *Lm = reinterpret_cast<const R *>(P.L), *Rm = reinterpret_cast<const R *>(P.R);
    R *out = reinterpret_cast<R *>(P.out);
    for (int m = blockIdx.x * 4 + wave; m < P.M; m += gridDim.x * 4) {
        R acc[SKINNY_MAX_N];
#pragma unroll
        for (int n = 0; n < SKINNY_MAX_N; n++) acc[n] = Ring<R>::zero();
        const R *row = Lm + (int64_t)m * K;
        for (int k = lane; k < K; k += 64) {
            const R a = ld(row, k);
#pragma unroll
            for (int n = 0; n < SKINNY_MAX_N; n++)
                if (n < N) acc[n] = mad(acc[n], a, ld(Rm, (int64_t)k * N + n));
        }
#pragma unroll
        for (int n = 0; n < SKINNY_MAX_N; n++) {
            if (n < N) {
                const R v = wave_sum(acc[n]);
                if (lane == 0) st(out, (int64_t)m * N + n, v);
            }
        }
    }
}

hipError_t launch_skinny(int eb, const SkinnyProb *probs_dev, int nprobs, int max_rows, hipStream_t st) {
    if (nprobs <= 0) return hipSuccess;
    int gx = (max_rows + 3) / 4;
    if (gx > 4096) gx = 4096;
    if (gx < 1) gx = 1;
    if (eb == 8) hipLaunchKernelGGL(k_skinny<r64>, dim3(gx, nprobs), dim3(256), 0, st, probs_dev, nprobs);
    else hipLaunchKernelGGL(k_skinny<u128>, dim3(gx, nprobs), dim3(256), 0, st, probs_dev, nprobs);
    return hipGetLastError();
}

}  // namespace ct
