// ct_kernels.hip -- the bandwidth-bound steps of the linear-layer hot path.
//
// The online phase touches every share array once, in three fused passes:
//   k_open_u   over K x N: opens U = Y - B (Fig. 7 online step 1), compresses
//              U and the tag shares of B along N (Fig. 7 step 6), and can
//              accumulate the batch tag check of U (Fig. 1);
//   k_row_pass over M x K, one wavefront per row: opens E = X - A, forms the
//              compact-tag products E U^c, E [tB^c]_p, [tA]_p U^c (Eq. (5)),
//              the folded operands A_0 + E and [tA]_p + [Delta]_p E of the
//              matrix-core products, or -- for layers with N <= 8 -- the whole
//              output (and SPDZ2k tag) products on the VALU, and can
//              accumulate the batch tag check of E;
//   k_post     over M x N, after the products: opens D = R - Z, writes the
//              optimistic tag (Pi_OptMAC) and compresses D, tag(R), tag(C)
//              along N (CompactTag), or accumulates the batch check of D
//              (SPDZ2k);
// then k_compact_final finishes Eq. (5) per row and can accumulate the compact
// check of D (Fig. 7 verification).  With F_CHECK the verification sums are
// formed by the passes that read the data anyway; without it ct_mac_check
// recomputes them with k_check_batch / k_check_compact.
//
// Every kernel serves all layers of a call: grid dimension y indexes layers
// (and sub-objects), dimension x strides over that layer's work.  Cross-
// workgroup sums use exact 128-bit atomics into zeroed accumulators.
#include "ct_device.h"

namespace ct {

constexpr int TPB = 256;
constexpr int WAVES = TPB / 64;
constexpr int SEGW = 512;  // elements per wavefront item of a long row

__device__ __forceinline__ u128 key_sum(const LayerDev &L) {
    const uint64_t lo = L.delta[0] + L.delta[1];
    return u128{lo, lo < L.delta[0] ? 1ull : 0ull};
}

__device__ __forceinline__ bool nz(u128 v) { return (v.lo | v.hi) != 0; }

static inline int grid_for(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}
static inline int grid_items(int64_t items) {  // one wavefront per item
    int64_t g = (items + WAVES - 1) / WAVES;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return (int)g;
}

// Adds each workgroup's NV sums (block-reduced) atomically into dst[0..NV).
template <int NV>
__device__ __forceinline__ void block_accumulate(u128 (&v)[NV], u128 *sh, u128 *dst) {
    block_sum<NV, WAVES>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++)
            if (nz(v[i])) atomic_add128(dst + i, v[i]);
    }
}

// Row sweep over an R x N matrix.  Rows of N <= 64 elements are reduced by
// groups of G = pow2ceil(N) lanes (64 / G rows per wavefront); longer rows
// are cut into items of SEGW elements, one wavefront each.  elem(r, c, v)
// accumulates into the NV row sums v; row_done(r, v) receives each item's sums
// (in the group leader lane) and must add them atomically.
template <int NV, typename Elem, typename RowDone>
__device__ __forceinline__ void row_sweep(int64_t rows, int64_t N, Elem elem, RowDone row_done) {
    const int lane = threadIdx.x & 63;
    const int64_t wave_id = (blockIdx.x * (int64_t)TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * TPB) >> 6;
    if (N <= 64) {
        int G = 1;
        while (G < N) G <<= 1;
        const int rpw = 64 / G;
        const int64_t items = (rows + rpw - 1) / rpw;
        for (int64_t it = wave_id; it < items; it += nwaves) {
            const int64_t r = it * rpw + lane / G;
            const int c = lane % G;
            u128 v[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = zero128();
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
            u128 v[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = zero128();
            for (int64_t c = c0 + lane; c < c1; c += 64) elem(r, c, v);
#pragma unroll
            for (int i = 0; i < NV; i++) v[i] = wave_sum(v[i]);
            if (lane == 0) row_done(r, v);
        }
    }
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
// Preprocessing of Fig. 7 / F_MAC Auth.  The lifts A~ and B~ are first written
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

// An input value of Z_{2^64}: the draw itself, or with in_bits in 1..63 a
// signed in_bits-bit integer (the draw's top bits, sign-extended) in two's
// complement.  Lifted with a zero upper limb.
__device__ __forceinline__ u128 input_lift(uint64_t draw, int in_bits) {
    if (in_bits <= 0 || in_bits >= 64) return u128{draw, 0};
    return u128{(uint64_t)((int64_t)draw >> (64 - in_bits)), 0};
}

// y = layer * NUM_OBJ + (object - 1); objects outside obj_mask, and R^f of
// layers with f = 0, are skipped.
__global__ void k_deal_auth(const LayerDev *__restrict__ Ls, int obj_mask) {
    const LayerDev &L = Ls[blockIdx.y / NUM_OBJ];
    const int obj = blockIdx.y % NUM_OBJ + 1;
    if (!((obj_mask >> obj) & 1) || (obj == OBJ_RF && L.f == 0)) return;
    int64_t n;
    u128 *const *v;
    u128 *const *t;
    switch (obj) {
        case OBJ_X: n = L.M * L.K; v = L.X; t = L.tX; break;
        case OBJ_Y: n = L.K * L.N; v = L.Y; t = L.tY; break;
        case OBJ_A: n = L.M * L.K; v = L.A; t = L.tA; break;
        case OBJ_B: n = L.K * L.N; v = L.B; t = L.tB; break;
        case OBJ_C: n = L.M * L.N; v = L.C; t = L.tC; break;
        case OBJ_R: n = L.M * L.N; v = L.R; t = L.tR; break;
        default: n = L.M * L.N; v = L.Rf; t = L.tRf; break;
    }
    u128 *v0 = v[0], *v1 = v[1], *t0 = t[0], *t1 = t[1];
    const uint64_t kv = L.key[K_VSH_X + obj - 1], kt = L.key[K_TSH_X + obj - 1];
    const u128 dsum = key_sum(L);
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        u128 lift;
        if (obj == OBJ_X) lift = input_lift(sdraw(L.key[K_LIFT_X], (uint64_t)e), L.in_bits);
        else if (obj == OBJ_Y) lift = input_lift(sdraw(L.key[K_LIFT_Y], (uint64_t)e), L.in_bits);
        else if (obj == OBJ_R) lift = sdraw128(L.key[K_LIFT_R], (uint64_t)e);
        else if (obj == OBJ_RF)  // R^f = (R mod 2^64) / 2^f, upper limb a fresh draw (Figs. 3 and 6)
            lift = u128{sdraw128(L.key[K_LIFT_R], (uint64_t)e).lo >> L.f, sdraw(L.key[K_LIFT_RF], (uint64_t)e)};
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
    hipLaunchKernelGGL(k_deal_auth, dim3(grid_for(max_elems), NUM_OBJ * n), dim3(TPB), 0, st, L, obj_mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------- zeroing
// what bit 0: the compressed vectors (cvec); bit 1: the check accumulators;
// bit 2: for layers with N <= SKINNY_MAX_N, [Z]_p = [C]_p (the row pass adds
// the products of each row segment atomically); bit 3: also [tZ]_p = [tC]_p.
__global__ void k_zero_acc(const LayerDev *__restrict__ Ls, int what) {
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t t0 = blockIdx.x * (int64_t)TPB + threadIdx.x, stride = (int64_t)gridDim.x * TPB;
    if (what & 1) {
        const int64_t n = 3 * L.K + 10 * L.M;
        for (int64_t e = t0; e < n; e += stride) st(L.cvec, e, zero128());
    }
    if ((what & 2) && blockIdx.x == 0 && threadIdx.x < ACC_PER_LAYER) st(L.acc, threadIdx.x, zero128());
    if ((what & 4) && L.N <= SKINNY_MAX_N) {
        const int64_t n = L.M * L.N;
        for (int64_t e = t0; e < n; e += stride) {
            st(L.Z[0], e, ld(L.C[0], e));
            st(L.Z[1], e, ld(L.C[1], e));
            if (what & 8) {
                st(L.tZ[0], e, ld(L.tC[0], e));
                st(L.tZ[1], e, ld(L.tC[1], e));
            }
        }
    }
}

hipError_t launch_zero_acc(const LayerDev *L, int n, int what, int64_t max_elems, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_acc, dim3((what & 5) ? grid_for(max_elems) : 1, n), dim3(TPB), 0, st, L, what);
    return hipGetLastError();
}

// Output arrays that receive split-K partial products start from their
// constant term: [Z]_p = [C]_p, and in SPDZ2k mode [tZ]_p = [tC]_p.  Layers
// whose products are formed in the row pass (N <= SKINNY_MAX_N) are skipped.
__global__ void k_copy_base(const LayerDev *__restrict__ Ls, int spdz) {
    const LayerDev &L = Ls[blockIdx.y >> 2];
    const int which = blockIdx.y & 3;  // 0,1: Z_p ; 2,3: tZ_p
    if ((which >= 2 && !spdz) || L.N <= SKINNY_MAX_N) return;
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

// ---------------------------------------------------------------- pass over K x N
// [U]_p = [Y]_p - [B]_p is party p's broadcast share and U = [U]_0 + [U]_1
// (Pi_BatchRec open).  CompactTag: U^c = U chi and [tB^c]_p = [tB]_p chi with
// chi_j drawn per column (Pi_Compress).  F_CHECK: the batch check sums of U,
// sum chi'_e ([tY]_p - [tB]_p) and sum chi'_e U_e.
__global__ __launch_bounds__(TPB) void k_open_u(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ u128 sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t K = L.K, N = L.N;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT;
    const CvecOff o = cvec_off(L.M, K);
    u128 chk[3] = {zero128(), zero128(), zero128()};
    const uint64_t kchi = L.key[K_CHI], kcu = L.key[K_CHI_U];
    auto elem = [&](int64_t r, int64_t c, u128 (&v)[3]) {
        const int64_t e = r * N + c;
        const u128 tb0 = ld(L.tB[0], e), tb1 = ld(L.tB[1], e);
        const u128 u = add(sub(ld(L.Y[0], e), ld(L.B[0], e)), sub(ld(L.Y[1], e), ld(L.B[1], e)));
        st(L.U, e, u);
        if (compact) {
            const uint64_t x = sdraw(kchi, (uint64_t)c);
            v[0] = mad64(v[0], u, x);
            v[1] = mad64(v[1], tb0, x);
            v[2] = mad64(v[2], tb1, x);
        }
        if (check) {
            const uint64_t x = sdraw(kcu, (uint64_t)e);
            chk[0] = mad64(chk[0], sub(ld(L.tY[0], e), tb0), x);
            chk[1] = mad64(chk[1], sub(ld(L.tY[1], e), tb1), x);
            chk[2] = mad64(chk[2], u, x);
        }
    };
    auto row_done = [&](int64_t r, u128 (&v)[3]) {
        if (compact) {
            atomic_add128(L.cvec + o.Uc + r, v[0]);
            atomic_add128(L.cvec + o.tBc0 + r, v[1]);
            atomic_add128(L.cvec + o.tBc1 + r, v[2]);
        }
    };
    row_sweep<3>(K, N, elem, row_done);
    if (check) block_accumulate<3>(chk, sh, L.acc + 3);
}

hipError_t launch_open_u(const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st) {
    hipLaunchKernelGGL(k_open_u, dim3(grid_items(max_items), n), dim3(TPB), 0, st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pass over M x K
// Work items are row segments of row_seg(M, K) elements, one wavefront each,
// lanes striding over k with coalesced loads; each item adds its row sums
// (compact-tag products, and the output products of skinny layers) to their
// destinations with exact 128-bit atomics.
template <int NS>
__device__ __forceinline__ void row_pass_body(const LayerDev &L, int flags, u128 (&chk)[3]) {
    const int lane = threadIdx.x & 63;
    const int64_t M = L.M, K = L.K, N = L.N;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT, spdz = flags & F_SPDZ;
    const bool skinny = NS > 0;
    const CvecOff o = cvec_off(M, K);
    const u128 *Uc = L.cvec + o.Uc, *tBc0 = L.cvec + o.tBc0, *tBc1 = L.cvec + o.tBc1;
    const uint64_t kce = L.key[K_CHI_E];
    const uint64_t d0 = L.delta[0], d1 = L.delta[1];
    u128 *AE0 = L.work, *tAE0 = L.work + M * K, *tAE1 = L.work + 2 * M * K;
    const int64_t seg = row_seg(M, K), items = M * ((K + seg - 1) / seg);
    const int64_t wave_id = (blockIdx.x * (int64_t)TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * TPB) >> 6;
    // segment-major order: the wavefronts in flight share one segment of k,
    // so the K-long vectors they read (U^c, [tB^c]_p; U, [B]_p of skinny
    // layers) stay in L2 while the M x K arrays stream through
    for (int64_t it = wave_id; it < items; it += nwaves) {
        const int64_t sg = it / M, m = it - sg * M, k0 = sg * seg;
        const int64_t k1 = k0 + seg < K ? k0 + seg : K;
        // compact: E U^c, E tB^c_0, E tB^c_1, tA_0 U^c, tA_1 U^c
        u128 cp[5] = {zero128(), zero128(), zero128(), zero128(), zero128()};
        // skinny: Z_0, Z_1 (and SPDZ2k tZ_0, tZ_1) row products per column
        u128 z0[NS > 0 ? NS : 1], z1[NS > 0 ? NS : 1], t0[NS > 0 ? NS : 1], t1[NS > 0 ? NS : 1];
#pragma unroll
        for (int j = 0; j < (NS > 0 ? NS : 1); j++) z0[j] = z1[j] = t0[j] = t1[j] = zero128();
        const int64_t rb = m * K;
        for (int64_t k = k0 + lane; k < k1; k += 64) {
            const int64_t e = rb + k;
            const u128 a0 = ld(L.A[0], e), a1 = ld(L.A[1], e);
            const u128 E = add(sub(ld(L.X[0], e), a0), sub(ld(L.X[1], e), a1));
            st(L.E, e, E);
            const bool need_ta = check || compact || spdz;
            u128 ta0 = zero128(), ta1 = zero128();
            if (need_ta) {
                ta0 = ld(L.tA[0], e);
                ta1 = ld(L.tA[1], e);
            }
            if (check) {
                const uint64_t x = sdraw(kce, (uint64_t)e);
                chk[0] = mad64(chk[0], sub(ld(L.tX[0], e), ta0), x);
                chk[1] = mad64(chk[1], sub(ld(L.tX[1], e), ta1), x);
                chk[2] = mad64(chk[2], E, x);
            }
            if (compact) {
                const u128 uc = ld(Uc, k);
                cp[0] = mad(cp[0], E, uc);
                cp[1] = mad(cp[1], E, ld(tBc0, k));
                cp[2] = mad(cp[2], E, ld(tBc1, k));
                cp[3] = mad(cp[3], ta0, uc);
                cp[4] = mad(cp[4], ta1, uc);
            }
            if constexpr (!skinny) {
                // folded left operands of the matrix-core products:
                //   [Z]_0 = [C]_0 + E [B]_0 + (A_0 + E) U,
                //   [tZ]_p = [tC]_p + E [tB]_p + ([tA]_p + [Delta]_p E) U
                st(AE0, e, add(a0, E));
                if (spdz) {
                    st(tAE0, e, add(ta0, mul64(E, d0)));
                    st(tAE1, e, add(ta1, mul64(E, d1)));
                }
            } else {
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    if (j < N) {
                        const int64_t kn = k * N + j;
                        const u128 u = ld(L.U, kn);
                        z0[j] = mad(mad(z0[j], E, add(ld(L.B[0], kn), u)), a0, u);
                        z1[j] = mad(mad(z1[j], E, ld(L.B[1], kn)), a1, u);
                        if (spdz) {
                            t0[j] = mad(mad(t0[j], E, add(ld(L.tB[0], kn), mul64(u, d0))), ta0, u);
                            t1[j] = mad(mad(t1[j], E, add(ld(L.tB[1], kn), mul64(u, d1))), ta1, u);
                        }
                    }
                }
            }
        }
        if (compact) {
#pragma unroll
            for (int i = 0; i < 5; i++) cp[i] = wave_sum(cp[i]);
            if (lane == 0) {
                // E U^c, and the partial compact tags (k_compact_final adds
                // [tC^c]_p and [Delta]_p E U^c)
                atomic_add128(L.cvec + o.EUc + m, cp[0]);
                atomic_add128(L.cvec + o.tZc0 + m, add(cp[1], cp[3]));
                atomic_add128(L.cvec + o.tZc1 + m, add(cp[2], cp[4]));
            }
        }
        if constexpr (skinny) {
#pragma unroll
            for (int j = 0; j < NS; j++) {
                if (j < N) {
                    z0[j] = wave_sum(z0[j]);
                    z1[j] = wave_sum(z1[j]);
                    if (spdz) {
                        t0[j] = wave_sum(t0[j]);
                        t1[j] = wave_sum(t1[j]);
                    }
                    if (lane == 0) {
                        // onto [Z]_p = [C]_p (and [tZ]_p = [tC]_p) set by k_zero_acc
                        const int64_t mn = m * N + j;
                        atomic_add128(L.Z[0] + mn, z0[j]);
                        atomic_add128(L.Z[1] + mn, z1[j]);
                        if (spdz) {
                            atomic_add128(L.tZ[0] + mn, t0[j]);
                            atomic_add128(L.tZ[1] + mn, t1[j]);
                        }
                    }
                }
            }
        }
    }
}

// Variant of the row pass a layer takes: 0 for matrix-core layers, else the
// smallest of 1, 2, 4, 8 that holds N.  Each variant is its own kernel so the
// register budget (and occupancy) of one does not limit the others.
__host__ __device__ inline int row_variant(int64_t N) {
    return N > SKINNY_MAX_N ? 0 : (N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : SKINNY_MAX_N)));
}

template <int NS>
__global__ __launch_bounds__(TPB) void k_row_pass(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ u128 sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    if (row_variant(L.N) != NS) return;
    u128 chk[3] = {zero128(), zero128(), zero128()};
    row_pass_body<NS>(L, flags, chk);
    if (flags & F_CHECK) block_accumulate<3>(chk, sh, L.acc + 0);
}

hipError_t launch_row_pass(const LayerDev *L, int n, int flags, int64_t max_items, int variants, hipStream_t st) {
    const dim3 g(grid_items(max_items), n), b(TPB);
    if (variants & (1 << 0)) hipLaunchKernelGGL(k_row_pass<0>, g, b, 0, st, L, flags);
    if (variants & (1 << 1)) hipLaunchKernelGGL(k_row_pass<1>, g, b, 0, st, L, flags);
    if (variants & (1 << 2)) hipLaunchKernelGGL(k_row_pass<2>, g, b, 0, st, L, flags);
    if (variants & (1 << 4)) hipLaunchKernelGGL(k_row_pass<4>, g, b, 0, st, L, flags);
    if (variants & (1 << 8)) hipLaunchKernelGGL(k_row_pass<SKINNY_MAX_N>, g, b, 0, st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pass over M x N
// D~ = ([R]_0 - [Z]_0) + ([R]_1 - [Z]_1) (Pi_OptMAC steps 1-2 / Pi_Truncation
// step 1).  CompactTag: [tZ]_p = [tR]_p - [Delta]_p D~ (Pi_OptMAC step 3) and
// the compressions D~^c, [tR^c]_p, [tC^c]_p (Fig. 7 step 6).  SPDZ2k with
// F_CHECK: the batch check sums of D with [tD]_p = [tR]_p - [tZ]_p.
// f > 0 (both protocols): the truncated output of OptMAC&Trunc (Fig. 6
// ExpandTrunc steps 2-4) / Pi_Truncation (Fig. 3 online step 2),
// [Z^f]_p = [R^f]_p - (D mod 2^64) / 2^f (party 0 subtracts the public term),
// [tZ^f]_p = [tR^f]_p - [Delta]_p (D mod 2^64) / 2^f.
__device__ __forceinline__ void truncate_out(const LayerDev &L, int64_t e, u128 D) {
    const uint64_t df = D.lo >> L.f;
    st(L.Zf[0], e, sub(ld(L.Rf[0], e), u128{df, 0}));
    st(L.Zf[1], e, ld(L.Rf[1], e));
    st(L.tZf[0], e, sub(ld(L.tRf[0], e), mul64(u128{L.delta[0], 0}, df)));
    st(L.tZf[1], e, sub(ld(L.tRf[1], e), mul64(u128{L.delta[1], 0}, df)));
}

__global__ __launch_bounds__(TPB) void k_post(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ u128 sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t M = L.M, N = L.N;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT;
    const CvecOff o = cvec_off(M, L.K);
    const uint64_t kchi = L.key[K_CHI], kcd = L.key[K_CHI_D];
    u128 chk[3] = {zero128(), zero128(), zero128()};
    if (compact) {
        auto elem = [&](int64_t r, int64_t c, u128 (&v)[5]) {
            const int64_t e = r * N + c;
            const u128 D = add(sub(ld(L.R[0], e), ld(L.Z[0], e)), sub(ld(L.R[1], e), ld(L.Z[1], e)));
            st(L.D, e, D);
            if (L.f > 0) truncate_out(L, e, D);
            const u128 tr0 = ld(L.tR[0], e), tr1 = ld(L.tR[1], e);
            st(L.tZ[0], e, sub(tr0, mul64(D, L.delta[0])));
            st(L.tZ[1], e, sub(tr1, mul64(D, L.delta[1])));
            const uint64_t x = sdraw(kchi, (uint64_t)c);
            v[0] = mad64(v[0], D, x);
            v[1] = mad64(v[1], tr0, x);
            v[2] = mad64(v[2], tr1, x);
            v[3] = mad64(v[3], ld(L.tC[0], e), x);
            v[4] = mad64(v[4], ld(L.tC[1], e), x);
        };
        auto row_done = [&](int64_t r, u128 (&v)[5]) {
            atomic_add128(L.cvec + o.Dc + r, v[0]);
            atomic_add128(L.cvec + o.tRc0 + r, v[1]);
            atomic_add128(L.cvec + o.tRc1 + r, v[2]);
            atomic_add128(L.cvec + o.tCc0 + r, v[3]);
            atomic_add128(L.cvec + o.tCc1 + r, v[4]);
        };
        row_sweep<5>(M, N, elem, row_done);
    } else {
        const int64_t n = M * N;
        for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
            const u128 z0 = ld(L.Z[0], e), z1 = ld(L.Z[1], e);
            const u128 D = add(sub(ld(L.R[0], e), z0), sub(ld(L.R[1], e), z1));
            st(L.D, e, D);
            if (L.f > 0) truncate_out(L, e, D);
            if (check) {
                const uint64_t x = sdraw(kcd, (uint64_t)e);
                chk[0] = mad64(chk[0], sub(ld(L.tR[0], e), ld(L.tZ[0], e)), x);
                chk[1] = mad64(chk[1], sub(ld(L.tR[1], e), ld(L.tZ[1], e)), x);
                chk[2] = mad64(chk[2], D, x);
            }
        }
        if (check) block_accumulate<3>(chk, sh, L.acc + 6);
    }
}

hipError_t launch_post(const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st) {
    hipLaunchKernelGGL(k_post, dim3(grid_items(max_items), n), dim3(TPB), 0, st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- compact tag
// Eq. (5) with the key on the public term, per row m:
//   [tZ^c]_p = [tC^c]_p + (E [tB^c]_p + [tA]_p U^c) + [Delta]_p (E U^c),
//   [tD^c]_p = [tR^c]_p - [tZ^c]_p.
// F_CHECK: the compact check of D (Fig. 7 verification steps 2-5) in the
// accumulator form of the batch checks,
//   acc6 = -sum chihat_i [tD^c]_{0,i}, acc7 = -sum chihat_i [tD^c]_{1,i},
//   acc8 = -sum chihat_i D^c_i,  so cs_p = acc_{6+p} - [Delta]_p acc8
//        = sum_i chihat_i ([Delta]_p D^c_i - [tD^c]_{p,i})   (mod 2^128).
__global__ __launch_bounds__(TPB) void k_compact_final(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ u128 sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t M = L.M;
    const CvecOff o = cvec_off(M, L.K);
    u128 *c = L.cvec;
    u128 v[3] = {zero128(), zero128(), zero128()};
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < M; i += (int64_t)gridDim.x * TPB) {
        const u128 eu = ld(c + o.EUc, i);
        const u128 z0 = add(add(ld(c + o.tCc0, i), ld(c + o.tZc0, i)), mul64(eu, L.delta[0]));
        const u128 z1 = add(add(ld(c + o.tCc1, i), ld(c + o.tZc1, i)), mul64(eu, L.delta[1]));
        const u128 dd0 = sub(ld(c + o.tRc0, i), z0), dd1 = sub(ld(c + o.tRc1, i), z1);
        st(c + o.tZc0, i, z0);
        st(c + o.tZc1, i, z1);
        st(c + o.tDc0, i, dd0);
        st(c + o.tDc1, i, dd1);
        if (flags & F_CHECK) {
            const uint64_t x = sdraw(L.key[K_CHIHAT], (uint64_t)i);
            v[0] = mad64(v[0], dd0, x);
            v[1] = mad64(v[1], dd1, x);
            v[2] = mad64(v[2], ld(c + o.Dc, i), x);
        }
    }
    if (flags & F_CHECK) {
#pragma unroll
        for (int i = 0; i < 3; i++) v[i] = sub(zero128(), v[i]);
        block_accumulate<3>(v, sh, L.acc + 6);
    }
}

hipError_t launch_compact_final(const LayerDev *L, int n, int flags, hipStream_t st) {
    hipLaunchKernelGGL(k_compact_final, dim3(4, n), dim3(TPB), 0, st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- MAC checks
// Standalone verification (ct_mac_check): Pi_BatchRec tag check (Fig. 1) of
// an opened W = P - Q with one public combiner chi'_e per element (drawn from
// the layer's stream; never stored):
//   acc0 = sum chi' ([tP]_0 - [tQ]_0),  acc1 = sum chi' ([tP]_1 - [tQ]_1),
//   accW = sum chi' W;   cs_p = acc_p - [Delta]_p accW   (mod 2^128).
// y = layer * 3 + which; which = 0: E (X, A), 1: U (Y, B), 2: D (R, Z).
__global__ __launch_bounds__(TPB) void k_check_batch(const LayerDev *__restrict__ Ls, int which_mask) {
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
    if (blockIdx.x * (int64_t)TPB >= n) return;  // no elements for this workgroup
    u128 v[3] = {zero128(), zero128(), zero128()};
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const uint64_t c = sdraw(key, (uint64_t)e);
        v[0] = mad64(v[0], sub(ld(tP0, e), ld(tQ0, e)), c);
        v[1] = mad64(v[1], sub(ld(tP1, e), ld(tQ1, e)), c);
        v[2] = mad64(v[2], ld(W, e), c);
    }
    block_accumulate<3>(v, sh, L.acc + 3 * which);
}

hipError_t launch_check_batch(const LayerDev *L, int n, int which_mask, int64_t max_elems, hipStream_t st) {
    int g = grid_for(max_elems);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_check_batch, dim3(g, 3 * n), dim3(TPB), 0, st, L, which_mask);
    return hipGetLastError();
}

// Standalone compact check of D from the stored compact vectors (same
// accumulator form as in k_compact_final).
__global__ __launch_bounds__(TPB) void k_check_compact(const LayerDev *__restrict__ Ls) {
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

hipError_t launch_finalize(const LayerDev *L, int n, ct_check_result *out, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, st, L, n, out);
    return hipGetLastError();
}

}  // namespace ct
