// ct_kernels.hip -- the bandwidth-bound steps of the linear-layer hot path:
// dealer fills, the openings of E, U and D, the optimistic tag, compression
// along N, the compact tag and the batch MAC checks.
//
// Every kernel takes the layer table and handles all layers of a call: grid
// dimension y indexes (layer, sub-object) and dimension x strides over the
// elements (or rows) of that layer.  Reductions go wavefront -> workgroup in
// registers and LDS, then one exact 128-bit atomic addition per workgroup.
#include "ct_device.h"

namespace ct {

constexpr int TPB = 256;
constexpr int WAVES = TPB / 64;

__device__ __forceinline__ u128 key_sum(const LayerDev &L) {
    const uint64_t lo = L.delta[0] + L.delta[1];
    return u128{lo, lo < L.delta[0] ? 1ull : 0ull};
}

static inline int grid_for(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

// ---------------------------------------------------------------- fill

__global__ void k_fill_zero(u128 *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
        st(p, i, zero128());
}

hipError_t launch_fill_zero(u128 *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n)), dim3(TPB), 0, st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- dealer
// Preprocessing of Fig. 6 / F_MAC Auth.  The lifts A~ and B~ are first written
// into party 1's buffers, the triple product C~ = A~ B~ is formed there by the
// ring GEMM, and k_deal_auth then splits every lift into value and tag shares.

__global__ void k_deal_lift(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y >> 1];
    const int which = blockIdx.y & 1;  // 0: A (M x K), 1: B (K x N)
    const int64_t n = which ? L.K * L.N : L.M * L.K;
    const uint64_t key = which ? L.key[K_LIFT_B] : L.key[K_LIFT_A];
    u128 *dst = which ? L.B[1] : L.A[1];
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB)
        st(dst, e, sdraw128(key, (uint64_t)e));
}

hipError_t launch_deal_lift(const LayerDev *L, int n, int64_t max_elems, hipStream_t st) {
    hipLaunchKernelGGL(k_deal_lift, dim3(grid_for(max_elems), 2 * n), dim3(TPB), 0, st, L);
    return hipGetLastError();
}

// y = layer * 6 + (object - 1); objects outside obj_mask are skipped.
__global__ void k_deal_auth(const LayerDev *__restrict__ Ls, int obj_mask) {
    const LayerDev &L = Ls[blockIdx.y / 6];
    const int obj = blockIdx.y % 6 + 1;
    if (!((obj_mask >> obj) & 1)) return;
    int64_t n;
    u128 **v, **t;
    switch (obj) {
        case OBJ_X: n = L.M * L.K; v = (u128 **)L.X; t = (u128 **)L.tX; break;
        case OBJ_Y: n = L.K * L.N; v = (u128 **)L.Y; t = (u128 **)L.tY; break;
        case OBJ_A: n = L.M * L.K; v = (u128 **)L.A; t = (u128 **)L.tA; break;
        case OBJ_B: n = L.K * L.N; v = (u128 **)L.B; t = (u128 **)L.tB; break;
        case OBJ_C: n = L.M * L.N; v = (u128 **)L.C; t = (u128 **)L.tC; break;
        default: n = L.M * L.N; v = (u128 **)L.R; t = (u128 **)L.tR; break;
    }
    u128 *v0 = v[0], *v1 = v[1], *t0 = t[0], *t1 = t[1];
    const uint64_t kv = L.key[K_VSH_X + obj - 1], kt = L.key[K_TSH_X + obj - 1];
    const u128 dsum = key_sum(L);
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        u128 lift;
        if (obj == OBJ_X) lift = u128{sdraw(L.key[K_LIFT_X], (uint64_t)e), 0};
        else if (obj == OBJ_Y) lift = u128{sdraw(L.key[K_LIFT_Y], (uint64_t)e), 0};
        else if (obj == OBJ_R) lift = sdraw128(L.key[K_LIFT_R], (uint64_t)e);
        else lift = ld(v1, e);  // A~, B~ or C~ left in party 1's buffer
        const u128 s0 = sdraw128(kv, (uint64_t)e);
        const u128 ts0 = sdraw128(kt, (uint64_t)e);
        const u128 tag = mul(lift, dsum);
        st(v0, e, s0);
        st(v1, e, sub(lift, s0));
        st(t0, e, ts0);
        st(t1, e, sub(tag, ts0));
    }
}

hipError_t launch_deal_auth(const LayerDev *L, int n, int obj_mask, int64_t max_elems, hipStream_t st) {
    hipLaunchKernelGGL(k_deal_auth, dim3(grid_for(max_elems), 6 * n), dim3(TPB), 0, st, L, obj_mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------- open E, U
// Fig. 6 online step 1 (Pi_BatchRec open): [W]_p = [P]_p - [Q]_p is each
// party's broadcast share and W = [W]_0 + [W]_1.

__global__ void k_open(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y >> 1];
    const int which = blockIdx.y & 1;  // 0: E = X - A, 1: U = Y - B
    const int64_t n = which ? L.K * L.N : L.M * L.K;
    const u128 *P0 = which ? L.Y[0] : L.X[0], *P1 = which ? L.Y[1] : L.X[1];
    const u128 *Q0 = which ? L.B[0] : L.A[0], *Q1 = which ? L.B[1] : L.A[1];
    u128 *W = which ? L.U : L.E;
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const u128 w0 = sub(ld(P0, e), ld(Q0, e));
        const u128 w1 = sub(ld(P1, e), ld(Q1, e));
        st(W, e, add(w0, w1));
    }
}

hipError_t launch_open(const LayerDev *L, int n, int64_t max_elems, hipStream_t st) {
    hipLaunchKernelGGL(k_open, dim3(grid_for(max_elems), 2 * n), dim3(TPB), 0, st, L);
    return hipGetLastError();
}

// Output arrays that receive split-K partial products start from their
// constant term: [Z]_p = [C]_p, and in SPDZ2k mode [tZ]_p = [tC]_p.
__global__ void k_copy_base(const LayerDev *__restrict__ Ls, int spdz) {
    const LayerDev &L = Ls[blockIdx.y >> 2];
    const int which = blockIdx.y & 3;  // 0,1: Z_p ; 2,3: tZ_p
    if (which >= 2 && !spdz) return;
    const int p = which & 1;
    const u128 *src = which >= 2 ? L.tC[p] : L.C[p];
    u128 *dst = which >= 2 ? L.tZ[p] : L.Z[p];
    const int64_t n = L.M * L.N;
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB)
        st(dst, e, ld(src, e));
}

hipError_t launch_copy_base(const LayerDev *L, int n, int mode, int64_t max_elems, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_base, dim3(grid_for(max_elems), 4 * n), dim3(TPB), 0, st, L,
                       mode == CT_MODE_SPDZ2K ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------- row reductions
// Rows of an R x N matrix are reduced against chi (Pi_Compress).  Rows with
// N <= SMALL_N are handled one per thread; longer rows are cut into segments
// of SEG elements, one workgroup per segment, combined by 128-bit atomics into
// the (pre-zeroed) destination.
constexpr int SMALL_N = 64;
constexpr int SEG = 4 * TPB;

__device__ __forceinline__ int64_t segs_per_row(int64_t N) { return (N + SEG - 1) / SEG; }

// Compress along N of the K x N matrices: U^c = U chi and [tB^c]_p = [tB]_p chi.
__global__ void k_compress_kn(const LayerDev *__restrict__ Ls) {
    __shared__ u128 sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t K = L.K, N = L.N;
    const CvecOff o = cvec_off(L.M, K);
    u128 *Uc = L.cvec + o.Uc, *tBc0 = L.cvec + o.tBc0, *tBc1 = L.cvec + o.tBc1;
    const uint64_t kchi = L.key[K_CHI];
    if (N <= SMALL_N) {
        for (int64_t r = blockIdx.x * (int64_t)TPB + threadIdx.x; r < K; r += (int64_t)gridDim.x * TPB) {
            u128 a = zero128(), b0 = zero128(), b1 = zero128();
            for (int64_t j = 0; j < N; j++) {
                const uint64_t c = sdraw(kchi, (uint64_t)j);
                const int64_t e = r * N + j;
                a = mad64(a, ld(L.U, e), c);
                b0 = mad64(b0, ld(L.tB[0], e), c);
                b1 = mad64(b1, ld(L.tB[1], e), c);
            }
            st(Uc, r, a);
            st(tBc0, r, b0);
            st(tBc1, r, b1);
        }
        return;
    }
    const int64_t spr = segs_per_row(N), nseg = K * spr;
    for (int64_t sgi = blockIdx.x; sgi < nseg; sgi += gridDim.x) {
        const int64_t r = sgi / spr, j0 = (sgi % spr) * SEG;
        u128 v[3] = {zero128(), zero128(), zero128()};
        for (int64_t j = j0 + threadIdx.x; j < j0 + SEG && j < N; j += TPB) {
            const uint64_t c = sdraw(kchi, (uint64_t)j);
            const int64_t e = r * N + j;
            v[0] = mad64(v[0], ld(L.U, e), c);
            v[1] = mad64(v[1], ld(L.tB[0], e), c);
            v[2] = mad64(v[2], ld(L.tB[1], e), c);
        }
        block_sum<3, WAVES>(v, sh);
        if (threadIdx.x == 0) {
            atomic_add128(Uc + r, v[0]);
            atomic_add128(tBc0 + r, v[1]);
            atomic_add128(tBc1 + r, v[2]);
        }
    }
}

static int row_grid(int64_t rows, int64_t max_segs) {
    int64_t g = max_segs;
    const int64_t gr = (rows + TPB - 1) / TPB;
    if (gr > g) g = gr;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_compress_kn(const LayerDev *L, int n, int64_t max_rows, int64_t max_segs, hipStream_t st) {
    hipLaunchKernelGGL(k_compress_kn, dim3(row_grid(max_rows, max_segs), n), dim3(TPB), 0, st, L);
    return hipGetLastError();
}

// COMPACT mode after the output GEMMs, per element of M x N:
//   D~ = ([R]_0 - [Z]_0) + ([R]_1 - [Z]_1)          (Pi_OptMAC steps 1-2)
//   [tZ]_p = [tR]_p - [Delta]_p D~                   (Pi_OptMAC step 3)
// and the compressions D~^c, [tR^c]_p, [tC^c]_p (Fig. 6 step 6) of the rows.
__device__ __forceinline__ u128 optmac_elem(const LayerDev &L, int64_t e) {
    const u128 d0 = sub(ld(L.R[0], e), ld(L.Z[0], e));
    const u128 d1 = sub(ld(L.R[1], e), ld(L.Z[1], e));
    const u128 D = add(d0, d1);
    st(L.D, e, D);
    return D;
}

__global__ void k_post_compact(const LayerDev *__restrict__ Ls) {
    __shared__ u128 sh[5 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t M = L.M, N = L.N;
    const CvecOff o = cvec_off(M, L.K);
    u128 *Dc = L.cvec + o.Dc, *tRc0 = L.cvec + o.tRc0, *tRc1 = L.cvec + o.tRc1;
    u128 *tCc0 = L.cvec + o.tCc0, *tCc1 = L.cvec + o.tCc1;
    const uint64_t kchi = L.key[K_CHI];
    auto elem = [&](int64_t e, uint64_t c, u128 (&v)[5]) {
        const u128 D = optmac_elem(L, e);
        const u128 tr0 = ld(L.tR[0], e), tr1 = ld(L.tR[1], e);
        st(L.tZ[0], e, sub(tr0, mul64(D, L.delta[0])));
        st(L.tZ[1], e, sub(tr1, mul64(D, L.delta[1])));
        v[0] = mad64(v[0], D, c);
        v[1] = mad64(v[1], tr0, c);
        v[2] = mad64(v[2], tr1, c);
        v[3] = mad64(v[3], ld(L.tC[0], e), c);
        v[4] = mad64(v[4], ld(L.tC[1], e), c);
    };
    if (N <= SMALL_N) {
        for (int64_t r = blockIdx.x * (int64_t)TPB + threadIdx.x; r < M; r += (int64_t)gridDim.x * TPB) {
            u128 v[5] = {zero128(), zero128(), zero128(), zero128(), zero128()};
            for (int64_t j = 0; j < N; j++) elem(r * N + j, sdraw(kchi, (uint64_t)j), v);
            st(Dc, r, v[0]);
            st(tRc0, r, v[1]);
            st(tRc1, r, v[2]);
            st(tCc0, r, v[3]);
            st(tCc1, r, v[4]);
        }
        return;
    }
    const int64_t spr = segs_per_row(N), nseg = M * spr;
    for (int64_t sgi = blockIdx.x; sgi < nseg; sgi += gridDim.x) {
        const int64_t r = sgi / spr, j0 = (sgi % spr) * SEG;
        u128 v[5] = {zero128(), zero128(), zero128(), zero128(), zero128()};
        for (int64_t j = j0 + threadIdx.x; j < j0 + SEG && j < N; j += TPB)
            elem(r * N + j, sdraw(kchi, (uint64_t)j), v);
        block_sum<5, WAVES>(v, sh);
        if (threadIdx.x == 0) {
            atomic_add128(Dc + r, v[0]);
            atomic_add128(tRc0 + r, v[1]);
            atomic_add128(tRc1 + r, v[2]);
            atomic_add128(tCc0 + r, v[3]);
            atomic_add128(tCc1 + r, v[4]);
        }
    }
}

hipError_t launch_post_compact(const LayerDev *L, int n, int64_t max_rows, int64_t max_segs, hipStream_t st) {
    hipLaunchKernelGGL(k_post_compact, dim3(row_grid(max_rows, max_segs), n), dim3(TPB), 0, st, L);
    return hipGetLastError();
}

// SPDZ2k mode: open D~ = sum_p ([R]_p - [Z]_p) (Pi_Truncation step 1).
__global__ void k_open_d(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t n = L.M * L.N;
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB)
        optmac_elem(L, e);
}

hipError_t launch_open_d(const LayerDev *L, int n, int64_t max_elems, hipStream_t st) {
    hipLaunchKernelGGL(k_open_d, dim3(grid_for(max_elems), n), dim3(TPB), 0, st, L);
    return hipGetLastError();
}

// ---------------------------------------------------------------- compact tag
// Eq. (7) with the key on the public term, one wavefront per row of E:
//   (E U^c)_m, [tZ^c]_p = [tC^c]_p + E [tB^c]_p + [tA]_p U^c + [Delta]_p (E U^c),
//   [tD^c]_p = [tR^c]_p - [tZ^c]_p.
__global__ void k_compact_tag(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t M = L.M, K = L.K;
    const CvecOff o = cvec_off(M, K);
    const u128 *Uc = L.cvec + o.Uc, *tBc0 = L.cvec + o.tBc0, *tBc1 = L.cvec + o.tBc1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t m = blockIdx.x * (int64_t)WAVES + wave; m < M; m += (int64_t)gridDim.x * WAVES) {
        u128 eu = zero128(), eb0 = zero128(), eb1 = zero128(), au0 = zero128(), au1 = zero128();
        const u128 *Er = L.E + m * K, *A0 = L.tA[0] + m * K, *A1 = L.tA[1] + m * K;
        for (int64_t k = lane; k < K; k += 64) {
            const u128 e = ld(Er, k), uc = ld(Uc, k);
            eu = mad(eu, e, uc);
            eb0 = mad(eb0, e, ld(tBc0, k));
            eb1 = mad(eb1, e, ld(tBc1, k));
            au0 = mad(au0, ld(A0, k), uc);
            au1 = mad(au1, ld(A1, k), uc);
        }
        eu = wave_sum(eu);
        eb0 = wave_sum(eb0);
        eb1 = wave_sum(eb1);
        au0 = wave_sum(au0);
        au1 = wave_sum(au1);
        if (lane == 0) {
            st(L.cvec + o.EUc, m, eu);
            u128 z0 = add(add(add(ld(L.cvec + o.tCc0, m), eb0), au0), mul64(eu, L.delta[0]));
            u128 z1 = add(add(add(ld(L.cvec + o.tCc1, m), eb1), au1), mul64(eu, L.delta[1]));
            st(L.cvec + o.tZc0, m, z0);
            st(L.cvec + o.tZc1, m, z1);
            st(L.cvec + o.tDc0, m, sub(ld(L.cvec + o.tRc0, m), z0));
            st(L.cvec + o.tDc1, m, sub(ld(L.cvec + o.tRc1, m), z1));
        }
    }
}

hipError_t launch_compact_tag(const LayerDev *L, int n, int64_t max_rows, hipStream_t st) {
    int64_t g = (max_rows + WAVES - 1) / WAVES;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_compact_tag, dim3((int)g, n), dim3(TPB), 0, st, L);
    return hipGetLastError();
}

// ---------------------------------------------------------------- zeroing
// what = 1: the compressed vectors accumulated by atomics; what = 2: the
// check accumulators.
__global__ void k_zero_acc(const LayerDev *__restrict__ Ls, int what) {
    const LayerDev &L = Ls[blockIdx.y];
    if (what == 1) {
        const int64_t n = 3 * L.K + 10 * L.M;
        for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB)
            st(L.cvec, e, zero128());
    } else if (blockIdx.x == 0 && threadIdx.x < ACC_PER_LAYER) {
        st(L.acc, threadIdx.x, zero128());
    }
}

hipError_t launch_zero_acc(const LayerDev *L, int n, int what, int64_t max_rows, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_acc, dim3(what == 1 ? grid_for(max_rows) : 1, n), dim3(TPB), 0, st, L, what);
    return hipGetLastError();
}

// ---------------------------------------------------------------- MAC checks
// Pi_BatchRec tag check (Fig. 1) of an opened W = P - Q with one public
// combiner chi'_e per element (drawn from the layer's stream; never stored):
//   acc0 = sum chi' ([tP]_0 - [tQ]_0),  acc1 = sum chi' ([tP]_1 - [tQ]_1),
//   accW = sum chi' W;   cs_p = acc_p - [Delta]_p accW   (mod 2^128).
// y = layer * 3 + which; which = 0: E (X, A), 1: U (Y, B), 2: D (R, Z).
__global__ void k_check_batch(const LayerDev *__restrict__ Ls, int which_mask) {
    __shared__ u128 sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y / 3];
    const int which = blockIdx.y % 3;
    if (!((which_mask >> which) & 1)) return;
    int64_t n;
    const u128 *tP0, *tP1, *tQ0, *tQ1, *W;
    uint64_t key;
    if (which == 0) {
        n = L.M * L.K; tP0 = L.tX[0]; tP1 = L.tX[1]; tQ0 = L.tA[0]; tQ1 = L.tA[1]; W = L.E; key = L.key[K_CHI_E];
    } else if (which == 1) {
        n = L.K * L.N; tP0 = L.tY[0]; tP1 = L.tY[1]; tQ0 = L.tB[0]; tQ1 = L.tB[1]; W = L.U; key = L.key[K_CHI_U];
    } else {
        n = L.M * L.N; tP0 = L.tR[0]; tP1 = L.tR[1]; tQ0 = L.tZ[0]; tQ1 = L.tZ[1]; W = L.D; key = L.key[K_CHI_D];
    }
    u128 v[3] = {zero128(), zero128(), zero128()};
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const uint64_t c = sdraw(key, (uint64_t)e);
        v[0] = mad64(v[0], sub(ld(tP0, e), ld(tQ0, e)), c);
        v[1] = mad64(v[1], sub(ld(tP1, e), ld(tQ1, e)), c);
        v[2] = mad64(v[2], ld(W, e), c);
    }
    block_sum<3, WAVES>(v, sh);
    if (threadIdx.x == 0) {
        u128 *acc = L.acc + 3 * which;
        atomic_add128(acc + 0, v[0]);
        atomic_add128(acc + 1, v[1]);
        atomic_add128(acc + 2, v[2]);
    }
}

hipError_t launch_check_batch(const LayerDev *L, int n, int which_mask, int64_t max_elems, hipStream_t st) {
    int g = grid_for(max_elems);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_check_batch, dim3(g, 3 * n), dim3(TPB), 0, st, L, which_mask);
    return hipGetLastError();
}

// Compact check of D (Fig. 6 verification steps 2-5), kept in the same
// accumulator form as the batch checks:
//   acc6 = -sum chihat_i [tD^c]_{0,i},  acc7 = -sum chihat_i [tD^c]_{1,i},
//   acc8 = -sum chihat_i D^c_i,   so  cs_p = acc_{6+p} - [Delta]_p acc8
//        = sum_i chihat_i ([Delta]_p D^c_i - [tD^c]_{p,i})   (mod 2^128).
__global__ void k_check_compact(const LayerDev *__restrict__ Ls) {
    __shared__ u128 sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t M = L.M;
    const CvecOff o = cvec_off(M, L.K);
    u128 v[3] = {zero128(), zero128(), zero128()};
    for (int64_t i = threadIdx.x; i < M; i += TPB) {
        const uint64_t c = sdraw(L.key[K_CHIHAT], (uint64_t)i);
        v[0] = mad64(v[0], ld(L.cvec + o.tDc0, i), c);
        v[1] = mad64(v[1], ld(L.cvec + o.tDc1, i), c);
        v[2] = mad64(v[2], ld(L.cvec + o.Dc, i), c);
    }
    block_sum<3, WAVES>(v, sh);
    if (threadIdx.x == 0) {
        st(L.acc, 6, sub(zero128(), v[0]));
        st(L.acc, 7, sub(zero128(), v[1]));
        st(L.acc, 8, sub(zero128(), v[2]));
    }
}

hipError_t launch_check_compact(const LayerDev *L, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_check_compact, dim3(1, n), dim3(TPB), 0, st, L);
    return hipGetLastError();
}

// cs[W][p] = acc[3W + p] - [Delta]_p acc[3W + 2]; accept iff every cs sum is 0.
__global__ void k_finalize(const LayerDev *__restrict__ Ls, int n, ct_check_result *out) {
    const int l = blockIdx.x * TPB + threadIdx.x;
    if (l >= n) return;
    const LayerDev &L = Ls[l];
    int ok = 1;
    ct_check_result r;
    for (int w = 0; w < 3; w++) {
        const u128 aw = ld(L.acc, 3 * w + 2);
        u128 c[2];
        for (int p = 0; p < 2; p++) {
            c[p] = sub(ld(L.acc, 3 * w + p), mul64(aw, L.delta[p]));
            r.cs[w][p].lo = c[p].lo;
            r.cs[w][p].hi = c[p].hi;
        }
        const u128 s = add(c[0], c[1]);
        if (s.lo != 0 || s.hi != 0) ok = 0;
    }
    r.accept = ok;
    r.reserved = 0;
    out[l] = r;
}

hipError_t launch_finalize(const LayerDev *L, int n, int mode, ct_check_result *out, hipStream_t st) {
    (void)mode;
    hipLaunchKernelGGL(k_finalize, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, st, L, n, out);
    return hipGetLastError();
}

}  // namespace ct
