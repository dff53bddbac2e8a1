// ct_sweep.h -- launch and reduction helpers shared by the kernel files of
// libcompacttag: element-type views of layer buffers, the key sum, launch
// sizing, block reductions into accumulators, and the row and column sweeps
// of a matrix with wavefront reductions.
#pragma once

#include "ct_device.h"

namespace ct {

constexpr int TPB = 256;
constexpr int WAVES = TPB / 64;
constexpr int SEGW = 512;  // elements per wavefront item of a long row

// The workgroup a stage body runs as: workgroup (x, y) of a grid with nx
// workgroups along x.  A stage kernel passes its own blockIdx and gridDim
// (hw_grid); the persistent launch runs the same bodies as workgroups of a
// grid of its choosing.
struct Grid {
    uint32_t x, y, nx;
};
__device__ __forceinline__ Grid hw_grid() { return Grid{blockIdx.x, blockIdx.y, gridDim.x}; }

// Buffers of a layer as elements of the context's ring (u128 for k = s = 64,
// r64 for k = s = 32).
template <class R>
__device__ __forceinline__ R *P(u128 *p) {
    return reinterpret_cast<R *>(p);
}

// Delta~ = [Delta]_0 + [Delta]_1 as an integer, as an element of the ring.
__device__ __forceinline__ void key_sum_to(const LayerDev &L, u128 &out) {
    const uint64_t lo = L.delta[0] + L.delta[1];
    out = u128{lo, lo < L.delta[0] ? 1ull : 0ull};
}
__device__ __forceinline__ void key_sum_to(const LayerDev &L, r64 &out) { out = r64{L.delta[0] + L.delta[1]}; }
// the sum over all np key shares, as an integer mod 2^{k+s}
__device__ __forceinline__ void key_sum_np_to(const LayerDev &L, u128 &out) {
    out = u128{0, 0};
    for (int p = 0; p < L.np; p++) {
        const uint64_t lo = out.lo + L.delta[p];
        out.hi += lo < out.lo ? 1ull : 0ull;
        out.lo = lo;
    }
}
__device__ __forceinline__ void key_sum_np_to(const LayerDev &L, r64 &out) {
    out = r64{0};
    for (int p = 0; p < L.np; p++) out.v += L.delta[p];
}
template <class R>
__device__ __forceinline__ R key_sum(const LayerDev &L) {
    R r;
    key_sum_to(L, r);
    return r;
}

// Launches kernel template KERN for the ring of element width eb bytes.
#define LAUNCH_RING(eb, KERN, grid, block, st, ...)                                   \
    do {                                                                              \
        if ((eb) == 8) hipLaunchKernelGGL(KERN<r64>, grid, block, 0, st, __VA_ARGS__);  \
        else hipLaunchKernelGGL(KERN<u128>, grid, block, 0, st, __VA_ARGS__);         \
    } while (0)

inline int grid_for(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}
inline int grid_items(int64_t items) {  // one wavefront per item
    int64_t g = (items + WAVES - 1) / WAVES;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return (int)g;
}

// The limb cells of a layer's row-pass copies (after its ACC_RP accumulators
// of the ring's element size).
template <class R>
__device__ __forceinline__ unsigned long long *rp_cells(const LayerDev &L) {
    return reinterpret_cast<unsigned long long *>(P<R>(L.acc) + ACC_RP);
}

// Adds each wavefront's NV sums (wave-reduced) into copy `copy` of the 4 NV
// limb cells at `cells`, without a workgroup barrier or waiting for the
// atomics: a wavefront that finishes early leaves at once.
template <int NV, class R>
__device__ __forceinline__ void wave_accumulate_limbs(R (&v)[NV], unsigned long long *cells) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const R s = wave_sum(v[i]);
        if ((threadIdx.x & 63) == 0) atomic_add_limbs(cells + 4 * i, s);
    }
}

// Adds each workgroup's NV sums (block-reduced) into the 4 NV limb cells of
// `cells` (atomic_add_limbs), without waiting for the atomics.
template <int NV, class R>
__device__ __forceinline__ void block_accumulate_limbs(R (&v)[NV], R *sh, unsigned long long *cells) {
    block_sum<NV, WAVES>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++) atomic_add_limbs(cells + 4 * i, v[i]);
    }
}

// Adds each workgroup's NV sums (block-reduced) atomically into dst[0..NV).
template <int NV, class R>
__device__ __forceinline__ void block_accumulate(R (&v)[NV], R *sh, R *dst) {
    block_sum<NV, WAVES>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++)
            if (Ring<R>::nonzero(v[i])) atomic_add128(dst + i, v[i]);
    }
}

// Row sweep over an R x N matrix by the workgroups of grid g.  Rows of N <= 64 elements are reduced by
// groups of G = pow2ceil(N) lanes (64 / G rows per wavefront); longer rows
// are cut into items of SEGW elements, one wavefront each.  elem(r, c, v)
// accumulates into the NV row sums v; row_done(r, v) receives each item's sums
// (in the group leader lane) and must add them atomically.
template <class R, int NV, typename Elem, typename RowDone>
__device__ __forceinline__ void row_sweep(const Grid &g, int64_t rows, int64_t N, Elem elem, RowDone row_done) {
    const int lane = threadIdx.x & 63;
    const int64_t wave_id = ((int64_t)g.x * TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)g.nx * TPB) >> 6;
    if (N <= 64) {
        int G = 1;
        while (G < N) G <<= 1;
        const int rpw = 64 / G;
        const int64_t items = (rows + rpw - 1) / rpw;
        for (int64_t it = wave_id; it < items; it += nwaves) {
            const int64_t r = it * rpw + lane / G;
            const int c = lane % G;
            R v[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = Ring<R>::zero();
            if (r < rows && c < N) elem(r, (int64_t)c, v);
            for (int m = G >> 1; m >= 1; m >>= 1) {
#pragma unroll
                for (int i = 0; i < NV; i++) v[i] = add(v[i], shfl_xor128(v[i], m));
            }
            if (c == 0 && r < rows) row_done(r, v);
        }
    } else {
        const int64_t segs = (N + SEGW - 1) / SEGW, items = rows * segs;
        for (int64_t it = wave_id; it < items; it += nwaves) {
            const int64_t r = it / segs, c0 = (it % segs) * SEGW;
            const int64_t c1 = c0 + SEGW < N ? c0 + SEGW : N;
            R v[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = Ring<R>::zero();
            for (int64_t c = c0 + lane; c < c1; c += 64) elem(r, c, v);
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = wave_sum(v[i]);
            if (lane == 0) row_done(r, v);
        }
    }
}

// Column sweep over an R x N matrix (sums down the columns), the mirror of
// row_sweep.  N <= 32: a wavefront covers 64 / G rows of G = pow2ceil(N)
// columns at a time (coalesced), takes rb such row groups per item and
// reduces over the lanes of one column; wider matrices give each lane a
// column and each item 64 columns of rb rows (rb = col_sweep_rb(rows)).
// elem(r, c, v) accumulates into the NV column sums v; col_done(c, v)
// receives each item's sums and must add them atomically.
template <class R, int NV, typename Elem, typename ColDone>
__device__ __forceinline__ void col_sweep(const Grid &g, int64_t rows, int64_t N, Elem elem, ColDone col_done) {
    const int lane = threadIdx.x & 63;
    const int64_t wave_id = ((int64_t)g.x * TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)g.nx * TPB) >> 6;
    const int64_t rb = col_sweep_rb(rows, N);
    if (N <= 32) {
        const int G = (int)col_sweep_group(N);
        const int rpw = 64 / G, c = lane % G;
        const int64_t per = (int64_t)rpw * rb, items = (rows + per - 1) / per;
        for (int64_t it = wave_id; it < items; it += nwaves) {
            R v[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = Ring<R>::zero();
            for (int64_t j = 0; j < rb; j++) {
                const int64_t r = it * per + (int64_t)j * rpw + lane / G;
                if (r < rows && c < N) elem(r, (int64_t)c, v);
            }
            for (int m = 32; m >= G; m >>= 1) {
#pragma unroll
                for (int i = 0; i < NV; i++) v[i] = add(v[i], shfl_xor128(v[i], m));
            }
            if (lane < G && c < N) col_done((int64_t)c, v);
        }
    } else {
        const int64_t chunks = (N + 63) / 64, items = chunks * ((rows + rb - 1) / rb);
        for (int64_t it = wave_id; it < items; it += nwaves) {
            const int64_t b = it / chunks, c = (it - b * chunks) * 64 + lane;
            const int64_t r0 = b * rb, r1 = r0 + rb < rows ? r0 + rb : rows;
            R v[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = Ring<R>::zero();
            if (c < N) {
                for (int64_t r = r0; r < r1; r++) elem(r, c, v);
                col_done(c, v);
            }
        }
    }
}

}  // namespace ct
