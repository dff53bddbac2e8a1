// ct_gemm.hip -- exact matrix products over Z_{2^128} for gfx950.
//
// The local products of Eqs. (2)-(3) (E*[B]_p, [A]_p*U, E*U and their tag
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
// Tile: 64 x 64 outputs per workgroup of 4 wavefronts (2 x 2), 32 x 32 per
// wavefront, K sliced by 32.  The operands of a slice are converted to digits
// by the loading threads and written to LDS as 16 digit planes per operand
// (plane d holds digit d of a 64 x 32 tile, 32 bytes per row or column, the
// two 16-byte halves swapped on every other group of 4 rows to spread LDS
// banks); two slices are double-buffered (128 KB).  A wavefront keeps the 16
// B digit fragments of its slice in registers and streams the A digits.
#include "ct_device.h"

namespace ct {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int PLANE = BM * BK;       // bytes per digit plane of a 64 x 32 tile
constexpr int OPBYTES = 16 * PLANE;  // 16 digit planes: 32 KB
constexpr int STAGE = 2 * OPBYTES;   // A and B: 64 KB

__device__ __forceinline__ void to_digits(u128 x, uint32_t (&w)[4]) {
    const uint64_t K = 0x8080808080808080ull;
    const uint64_t lo = x.lo + K;
    const uint64_t hi = x.hi + K + (lo < K ? 1ull : 0ull);
    w[0] = (uint32_t)(lo ^ K);
    w[1] = (uint32_t)((lo ^ K) >> 32);
    w[2] = (uint32_t)(hi ^ K);
    w[3] = (uint32_t)((hi ^ K) >> 32);
}

// byte offset of (row, k) inside one digit plane (k multiple of 8 or 16)
__device__ __forceinline__ int plane_off(int row, int k) {
    const int chunk = k >> 4;
    return row * BK + (((chunk ^ (row >> 2)) & 1) << 4) + (k & 15);
}

// Transposes digits of 8 consecutive-k elements into 16 planes of 8 bytes and
// writes them at base + d * PLANE + off.
__device__ __forceinline__ void write_planes(uint8_t *base, int off, const uint32_t (&w)[8][4]) {
#pragma unroll
    for (int q = 0; q < 4; q++) {  // dword q holds digits 4q .. 4q+3
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

__device__ __forceinline__ void gemm_tile(const GemmProb &P, int tm, int tn, int split, uint8_t *smem) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = P.M, N = P.N, K = P.K;
    const int m0 = tm * BM, n0 = tn * BN;
    const int s_begin = split * P.steps_per_split;
    const int s_end = min(s_begin + P.steps_per_split, P.nsteps);

    // loader coordinates: A thread -> (row, 8 consecutive k); B thread -> (col, 8 consecutive k)
    const int ar = tid >> 2, akk = (tid & 3) * 8;
    const int bc = tid & 63, bkk = (tid >> 6) * 8;
    const int a_off = plane_off(ar, akk);
    const int b_off = plane_off(bc, bkk);

    v16i acc[16];
#pragma unroll
    for (int t = 0; t < 16; t++) acc[t] = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

    // Branch-free operand loads: buffer loads whose out-of-range offset returns
    // zero.  Descriptors are based at the tile's first row (A) and at the K
    // slice's first row (B), so 32-bit offsets suffice for any matrix size.
    constexpr uint32_t OOB = 0x80000000u;
    auto rsrc = [](const u128 *base, int64_t bytes) {
        const int32_t nrec = bytes > 0x7FFFFFF0LL ? 0x7FFFFFF0 : (int32_t)bytes;
        return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, nrec, 0x00020000);
    };
    const bool arow_ok = m0 + ar < M;
    const bool bcol_ok = n0 + bc < N;
    v4i ra[8], rb[8];
    auto gload = [&](int step) {
        const int seg = step >= P.ksteps_seg ? 1 : 0;
        const int kb = (step - seg * P.ksteps_seg) * BK;
        const u128 *Ls = seg ? P.L2 : P.L1;
        const u128 *Rs = seg ? P.R2 : P.R1;
        const auto ra_rs = rsrc(Ls + (int64_t)m0 * K, (int64_t)(M - m0) * K * 16);
        const auto rb_rs = rsrc(Rs + (int64_t)kb * N, (int64_t)(K - kb) * N * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = kb + akk + j;
            const uint32_t off = (arow_ok && k < K) ? (uint32_t)(ar * K + k) * 16u : OOB;
            ra[j] = __builtin_amdgcn_raw_buffer_load_b128(ra_rs, off, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int kk = bkk + j;
            const uint32_t off = (bcol_ok && kb + kk < K) ? (uint32_t)(kk * N + n0 + bc) * 16u : OOB;
            rb[j] = __builtin_amdgcn_raw_buffer_load_b128(rb_rs, off, 0, 0);
        }
    };
    auto as128 = [](v4i v) {
        return u128{(uint64_t)(uint32_t)v[0] | ((uint64_t)(uint32_t)v[1] << 32),
                    (uint64_t)(uint32_t)v[2] | ((uint64_t)(uint32_t)v[3] << 32)};
    };
    auto lstore = [&](uint8_t *stage) {
        uint32_t w[8][4];
#pragma unroll
        for (int j = 0; j < 8; j++) to_digits(as128(ra[j]), w[j]);
        write_planes(stage, a_off, w);
#pragma unroll
        for (int j = 0; j < 8; j++) to_digits(as128(rb[j]), w[j]);
        write_planes(stage + OPBYTES, b_off, w);
    };

    // MFMA-side fragment offsets (lane -> row/col lane%32, k half lane/32)
    const int chunk = lane >> 5;
    const int arow = wm * 32 + (lane & 31);
    const int brow = wn * 32 + (lane & 31);
    const int a_frag = arow * BK + (((chunk ^ (arow >> 2)) & 1) << 4);
    const int b_frag = brow * BK + (((chunk ^ (brow >> 2)) & 1) << 4);

    if (s_begin < s_end) {
        gload(s_begin);
        lstore(smem);
    }
    __syncthreads();
    for (int s = s_begin; s < s_end; s++) {
        const int buf = (s - s_begin) & 1;
        const uint8_t *cur = smem + buf * STAGE;
        uint8_t *nxt = smem + (buf ^ 1) * STAGE;
        const bool more = s + 1 < s_end;
        if (more) gload(s + 1);

        v4i b[16];
#pragma unroll
        for (int j = 0; j < 16; j++) b[j] = *reinterpret_cast<const v4i *>(cur + OPBYTES + j * PLANE + b_frag);
        v4i a = *reinterpret_cast<const v4i *>(cur + a_frag);
#pragma unroll
        for (int i = 0; i < 16; i++) {
            // prefetch the next A digit plane while this one's products issue
            const v4i an = *reinterpret_cast<const v4i *>(cur + ((i + 1) & 15) * PLANE + a_frag);
#pragma unroll
            for (int j = 0; j < 16 - i; j++)
                acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b[j], acc[i + j], 0, 0, 0);
            a = an;
        }

        if (more) lstore(nxt);
        __syncthreads();
    }

    // epilogue: 32x32 accumulator layout -- lane l, register r holds
    // row 8*(r/4) + 4*(l/32) + r%4, column l%32 of the wavefront's tile.
    const int col = n0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int row = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        u128 v = zero128();
        combine<0>(acc, r, v);
        if (row < M && col < N) {
            const int64_t idx = (int64_t)row * N + col;
            if (P.accumulate) {
                atomic_add128(P.out + idx, v);
            } else {
                if (P.base) v = add(v, ld(P.base, idx));
                st(P.out, idx, v);
            }
        }
    }
}

__global__ __launch_bounds__(256, 1) void k_ring_gemm(const GemmProb *__restrict__ probs, int nprobs,
                                                      int total_tiles) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[2 * STAGE];
    for (int t = blockIdx.x; t < total_tiles; t += gridDim.x) {
        int lo = 0, hi = nprobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (probs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        const GemmProb P = probs[lo];
        int local = t - P.tile_begin;
        const int split = local % P.splits;
        local /= P.splits;
        const int tn = local % P.tiles_n, tm = local / P.tiles_n;
        gemm_tile(P, tm, tn, split, smem);
        __syncthreads();
    }
}

hipError_t launch_gemm(const GemmProb *probs_dev, int nprobs, int total_tiles, int grid, hipStream_t st) {
    if (nprobs <= 0 || total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ring_gemm, dim3(grid), dim3(256), 0, st, probs_dev, nprobs, total_tiles);
    return hipGetLastError();
}

// ---------------------------------------------------------------- skinny
// The dealer's triple product C~ = A~ B~ for layers with few output columns
// (N <= SKINNY_MAX_N, e.g. a classifier layer at batch 1) is a bandwidth-bound
// row-times-matrix product: one wavefront per output row, lanes striding over
// K with coalesced 16-byte loads, 128-bit VALU multiply-adds, a wavefront
// reduction per column.  (The online phase forms these products inside its
// pass over E.)
__global__ __launch_bounds__(256) void k_skinny(const GemmProb *__restrict__ probs, int nprobs) {
    const GemmProb P = probs[blockIdx.y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int N = P.N, K = P.K;
    for (int m = blockIdx.x * 4 + wave; m < P.M; m += gridDim.x * 4) {
        u128 acc[SKINNY_MAX_N];
#pragma unroll
        for (int n = 0; n < SKINNY_MAX_N; n++) acc[n] = zero128();
        for (int seg = 0; seg < (P.L2 ? 2 : 1); seg++) {
            const u128 *Ls = seg ? P.L2 : P.L1;
            const u128 *Rs = seg ? P.R2 : P.R1;
            const u128 *row = Ls + (int64_t)m * K;
            for (int k = lane; k < K; k += 64) {
                const u128 a = ld(row, k);
#pragma unroll
                for (int n = 0; n < SKINNY_MAX_N; n++) {
                    if (n < N) {
                        acc[n] = mad(acc[n], a, ld(Rs, (int64_t)k * N + n));
                    }
                }
            }
        }
#pragma unroll
        for (int n = 0; n < SKINNY_MAX_N; n++) {
            if (n < N) {
                u128 v = wave_sum(acc[n]);
                if (lane == 0) {
                    const int64_t idx = (int64_t)m * N + n;
                    if (P.accumulate) {
                        atomic_add128(P.out + idx, v);
                    } else {
                        if (P.base) v = add(v, ld(P.base, idx));
                        st(P.out, idx, v);
                    }
                }
            }
        }
    }
}

hipError_t launch_skinny(const GemmProb *probs_dev, int nprobs, int max_rows, hipStream_t st) {
    if (nprobs <= 0) return hipSuccess;
    int gx = (max_rows + 3) / 4;
    if (gx > 4096) gx = 4096;
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(k_skinny, dim3(gx, nprobs), dim3(256), 0, st, probs_dev, nprobs);
    return hipGetLastError();
}

}  // namespace ct
