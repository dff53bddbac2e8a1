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
// Layers compressed along M take k_row_pass_cm (column sums of E and [tA]_p),
// a column sweep in k_post and k_col_tag (the compact-tag products over
// K x N).  Convolution layers open U on their input's elements in k_open_u
// and compress their implicit im2col matrices in k_conv_compress.  Two-party
// matrix-core layers that are not convolutions open U in k_open_pack
// (ct_gemm.hip), which also writes their right operands' digit tiles.
//
// Every kernel serves all layers of a call: grid dimension y indexes layers
// (and sub-objects), dimension x strides over that layer's work.  Cross-
// workgroup sums use exact 128-bit atomics into zeroed accumulators.
#include "ct_passes.h"

namespace ct {

// ---------------------------------------------------------------- fill

template <class R>
__global__ void k_fill_zero(u128 *p_, int64_t n) {
    R *p = P<R>(p_);
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
        st(p, i, Ring<R>::zero());
}

hipError_t launch_fill_zero(int eb, u128 *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    LAUNCH_RING(eb, k_fill_zero, dim3(grid_for(n)), dim3(TPB), st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- dealer
// Preprocessing of Fig. 7 / F_MAC Auth.  The lifts A~ and B~ are first written
// into party 1's buffers, the triple product C~ = A~ B~ is formed there by the
// ring GEMM, and k_deal_auth then splits every lift into value and tag shares.

template <class R>
__global__ void k_deal_lift(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y >> 1];
    const int which = blockIdx.y & 1;  // 0: A (M x K), 1: B (K x N, or a convolution input's shape)
    const int64_t n = which ? L.nr : L.M * L.K;
    const uint64_t key = which ? L.key[K_LIFT_B] : L.key[K_LIFT_A];
    R *dst = which ? P<R>(L.B[1]) : P<R>(L.A[1]);
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB)
        st(dst, e, Ring<R>::draw(key, (uint64_t)e));
}

hipError_t launch_deal_lift(int eb, const LayerDev *L, int n, int64_t max_elems, hipStream_t st) {
    LAUNCH_RING(eb, k_deal_lift, dim3(grid_for(max_elems), 2 * n), dim3(TPB), st, L);
    return hipGetLastError();
}

// Inputs are values of Z_{2^k} (uniform, or signed in_bits-bit integers in
// two's complement: Ring<R>::input) lifted with zero upper bits.

// y = layer * NUM_OBJ + (object - 1); objects outside obj_mask, and R^f of
// layers with f = 0, are skipped.
template <class R>
__global__ void k_deal_auth(const LayerDev *__restrict__ Ls, int obj_mask) {
    const LayerDev &L = Ls[blockIdx.y / NUM_OBJ];
    const int obj = blockIdx.y % NUM_OBJ + 1;
    if (!((obj_mask >> obj) & 1) || (obj == OBJ_RF && L.f == 0)) return;
    int64_t n;
    u128 *const *v;
    u128 *const *t;
    switch (obj) {
        case OBJ_X: n = L.M * L.K; v = L.X; t = L.tX; break;
        case OBJ_Y: n = L.nr; v = L.Y; t = L.tY; break;
        case OBJ_A: n = L.M * L.K; v = L.A; t = L.tA; break;
        case OBJ_B: n = L.nr; v = L.B; t = L.tB; break;
        case OBJ_C: n = L.M * L.N; v = L.C; t = L.tC; break;
        case OBJ_R: n = L.M * L.N; v = L.R; t = L.tR; break;
        default: n = L.M * L.N; v = L.Rf; t = L.tRf; break;
    }
    R *v0 = P<R>(v[0]), *v1 = P<R>(v[1]), *t0 = P<R>(t[0]), *t1 = P<R>(t[1]);
    const uint64_t kv = L.key[K_VSH_X + obj - 1], kt = L.key[K_TSH_X + obj - 1];
    const R dsum = key_sum<R>(L);
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        R lift;
        if (obj == OBJ_X) lift = Ring<R>::input(sdraw(L.key[K_LIFT_X], (uint64_t)e), L.in_bits);
        else if (obj == OBJ_Y) lift = Ring<R>::input(sdraw(L.key[K_LIFT_Y], (uint64_t)e), L.in_bits);
        else if (obj == OBJ_R) lift = Ring<R>::draw(L.key[K_LIFT_R], (uint64_t)e);
        else if (obj == OBJ_RF)  // R^f = (R mod 2^k) / 2^f, upper part a fresh draw (Figs. 3 and 6)
            lift = Ring<R>::lift(Ring<R>::mod_k(Ring<R>::draw(L.key[K_LIFT_R], (uint64_t)e)) >> L.f,
                                 Ring<R>::mod_s(sdraw(L.key[K_LIFT_RF], (uint64_t)e)));
        else lift = ld(v1, e);  // A~, B~ or C~ left in party 1's buffer
        const R s0 = Ring<R>::draw(kv, (uint64_t)e);
        const R ts0 = Ring<R>::draw(kt, (uint64_t)e);
        const R tag = mul(lift, dsum);
        st(v0, e, s0);
        st(v1, e, sub(lift, s0));
        st(t0, e, ts0);
        st(t1, e, sub(tag, ts0));
    }
}

hipError_t launch_deal_auth(int eb, const LayerDev *L, int n, int obj_mask, int64_t max_elems, hipStream_t st) {
    LAUNCH_RING(eb, k_deal_auth, dim3(grid_for(max_elems), NUM_OBJ * n), dim3(TPB), st, L, obj_mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------- zeroing
// what bit 0: the compressed vectors (cvec); bit 1: the check accumulators;
// bit 2: for layers with N <= SKINNY_MAX_N, [Z]_p = [C]_p (the row pass adds
// the products of each row segment atomically); bit 3: also [tZ]_p = [tC]_p.
template <class R>
__global__ void k_zero_acc(const LayerDev *__restrict__ Ls, int what) {
    zero_acc_body<R>(Ls, what, hw_grid());
}

hipError_t launch_zero_acc(int eb, const LayerDev *L, int n, int what, int64_t max_elems, hipStream_t st) {
    LAUNCH_RING(eb, k_zero_acc, dim3((what & 5) ? grid_for(max_elems) : 1, n), dim3(TPB), st, L, what);
    return hipGetLastError();
}

// Products whose K range is split add their partial results atomically onto
// the output, which first receives the product's constant term: [Z]_p = [C]_p
// (SPDZ2k also [tZ]_p = [tC]_p).  Only the split products are copied; the
// others add the constant term in the product's epilogue.
template <class R>
__global__ void k_prob_base(const GemmProb *__restrict__ probs) {
    prob_base_body<R>(probs, hw_grid());
}

hipError_t launch_prob_base(int eb, const GemmProb *probs, int nprobs, int64_t max_mn, hipStream_t st) {
    if (nprobs <= 0) return hipSuccess;
    LAUNCH_RING(eb, k_prob_base, dim3(grid_for(max_mn), nprobs), dim3(TPB), st, probs);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pass over K x N
// [U]_p = [Y]_p - [B]_p is party p's broadcast share and U = [U]_0 + [U]_1
// (Pi_BatchRec open).  CompactTag: U^c = U chi and [tB^c]_p = [tB]_p chi with
// chi_j drawn per column (Pi_Compress).  F_CHECK: the batch check sums of U,
// sum chi'_e ([tY]_p - [tB]_p) and sum chi'_e U_e.
template <class R>
__global__ __launch_bounds__(TPB) void k_open_u(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ R sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    if (L.fo) return;  // opened by k_open_pack
    const int64_t K = L.K, N = L.N;
    // a layer compressed along M has no K-long compressions of U and [tB]_p
    const bool check = flags & F_CHECK, compact = (flags & F_COMPACT) && !L.cm;
    const CvecOff o = cvec_off(L.M, K);
    R chk[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    const uint64_t kchi = L.key[K_CHI], kcu = L.key[K_CHI_U];
    auto elem = [&](int64_t r, int64_t c, R (&v)[3]) {
        const int64_t e = r * N + c;
        const R tb0 = ld(P<R>(L.tB[0]), e), tb1 = ld(P<R>(L.tB[1]), e);
        const R u = add(sub(ld(P<R>(L.Y[0]), e), ld(P<R>(L.B[0]), e)), sub(ld(P<R>(L.Y[1]), e), ld(P<R>(L.B[1]), e)));
        st(P<R>(L.U), e, u);
        if (compact) {
            const uint64_t x = Ring<R>::mod_s(sdraw(kchi, (uint64_t)c));
            v[0] = mad64(v[0], u, x);
            v[1] = mad64(v[1], tb0, x);
            v[2] = mad64(v[2], tb1, x);
        }
        if (check) {
            const uint64_t x = Ring<R>::mod_s(sdraw(kcu, (uint64_t)e));
            chk[0] = mad64(chk[0], sub(ld(P<R>(L.tY[0]), e), tb0), x);
            chk[1] = mad64(chk[1], sub(ld(P<R>(L.tY[1]), e), tb1), x);
            chk[2] = mad64(chk[2], u, x);
        }
    };
    auto row_done = [&](int64_t r, R (&v)[3]) {
        if (compact) add_cells<3>(P<R>(L.cvec), {o.Uc, o.tBc0, o.tBc1}, r, v);
    };
    if (L.cv.on) {
        // a convolution opens U on the input's elements; their compression
        // along N (an implicit im2col) is k_conv_compress
        for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < L.nr; e += (int64_t)gridDim.x * TPB) {
            const R tb0 = ld(P<R>(L.tB[0]), e), tb1 = ld(P<R>(L.tB[1]), e);
            const R u = add(sub(ld(P<R>(L.Y[0]), e), ld(P<R>(L.B[0]), e)), sub(ld(P<R>(L.Y[1]), e), ld(P<R>(L.B[1]), e)));
            st(P<R>(L.U), e, u);
            if (check) {
                const uint64_t x = Ring<R>::mod_s(sdraw(kcu, (uint64_t)e));
                chk[0] = mad64(chk[0], sub(ld(P<R>(L.tY[0]), e), tb0), x);
                chk[1] = mad64(chk[1], sub(ld(P<R>(L.tY[1]), e), tb1), x);
                chk[2] = mad64(chk[2], u, x);
            }
        }
    } else {
        row_sweep<R, 3>(hw_grid(), K, N, elem, row_done);
    }
    if (check) block_accumulate<3>(chk, sh, P<R>(L.acc) + 3);
}

// Compression along N of a convolution's implicit im2col matrices (Pi_Compress,
// Fig. 4, with the right operand of Eq. (4)): for row k = (c, dy, dx),
//   U^c_k = sum_n chi_n U[c, y s + dy - p, x s + dx - p]   (n = y Wo + x),
// and [tB^c]_p alike -- a k x k correlation of the input with chi laid out as
// an Ho x Wo image.  Work items are (channel c, segment of CONV_SEG positions
// n), one workgroup of CONV_WAVES wavefronts each; the wavefronts share out
// the k x k rows (c, dy, dx) of the channel (three each for a 3 x 3 window),
// so the input rows under the segment and the window's halo are fetched once
// into the compute unit's caches and read there by all k^2 rows.  (Rows
// taken as independent wavefront items went round-robin over the XCDs, each
// of whose L2s fetched the same input lines: 6.5x the input's bytes.)
constexpr int CONV_SEG = 512;
constexpr int CONV_WAVES = 3;
template <class R>
__global__ __launch_bounds__(TPB) void k_conv_compress(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y];
    if (!L.cv.on || L.cm) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const CvecOff o = cvec_off(L.M, L.K);
    const uint64_t kchi = L.key[K_CHI];
    const int N = (int)L.N, kk = L.cv.k * L.cv.k;
    const int segs = (N + CONV_SEG - 1) / CONV_SEG;
    const int64_t items = (int64_t)L.cv.c * segs;
    constexpr int J = CONV_SEG / 64;  // positions per lane and segment
    R *cv = P<R>(L.cvec);
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int ch = (int)(it / segs), n0 = (int)(it - (int64_t)ch * segs) * CONV_SEG;
        uint64_t chi[J];
#pragma unroll
        for (int j = 0; j < J; j++) {
            const int n = n0 + 64 * j + lane;
            chi[j] = n < N ? Ring<R>::mod_s(sdraw(kchi, (uint64_t)n)) : 0;
        }
        for (int t = wave; t < kk; t += CONV_WAVES) {
            const int32_t k = ch * kk + t;
            R v[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
#pragma unroll
            for (int j = 0; j < J; j++) {
                const int n = n0 + 64 * j + lane;
                const int64_t g = n < N ? conv_src(L.cv, k, n) : -1;
                if (g >= 0) {
                    v[0] = mad64(v[0], ld(P<R>(L.U), g), chi[j]);
                    v[1] = mad64(v[1], ld(P<R>(L.tB[0]), g), chi[j]);
                    v[2] = mad64(v[2], ld(P<R>(L.tB[1]), g), chi[j]);
                }
            }
#pragma unroll
            for (int i = 0; i < 3; i++) v[i] = wave_sum(v[i]);
            if (lane == 0) {
                R *const cell[3] = {cv + o.Uc + k, cv + o.tBc0 + k, cv + o.tBc1 + k};
                const bool ok[3] = {true, true, true};
                atomic_add128_n<3>(cell, v, ok);
            }
        }
    }
}

hipError_t launch_conv_compress(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st) {
    // one workgroup per (channel, segment) item
    const int gx = (int)std::min<int64_t>(std::max<int64_t>(max_items, 1), 16384);
    LAUNCH_RING(eb, k_conv_compress, dim3(gx, n), dim3(64 * CONV_WAVES), st, L);
    return hipGetLastError();
}

hipError_t launch_open_u(int eb, const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st) {
    LAUNCH_RING(eb, k_open_u, dim3(grid_items(max_items), n), dim3(TPB), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pass over M x K
// Work items are row segments of row_seg(M, K) elements, one wavefront each,
// lanes striding over k with coalesced loads; each item adds its row sums
// (compact-tag products, and the output products of skinny layers) to their
// destinations with exact 128-bit atomics (row_pass_body, ct_passes.h).
// The row pass of a CompactTag layer compressed along M (chi of length M):
// besides opening E, checking it and (N <= SKINNY_MAX_N) forming the output
// products, it compresses E and [tA]_p down the columns,
//   E^c_k = sum_m chi_m E_mk,  [tA^c]_p,k = sum_m chi_m [tA]_p,mk  (Fig. 4 along M).
// Work items are strips of cm_cw(N) * 64 columns over CM_RB rows, ordered
// row-block-major so that concurrent wavefronts read neighbouring columns of
// the same rows and add their column sums to different addresses.
template <class R, int NS>
__device__ __forceinline__ void row_pass_cm(const LayerDev &L, int flags, R (&chk)[3]) {
    const int lane = threadIdx.x & 63;
    const int64_t M = L.M, K = L.K, N = L.N;
    const bool check = flags & F_CHECK;
    const CvecOff o = cvec_off(N, K);
    const uint64_t kce = L.key[K_CHI_E], kchi = L.key[K_CHI];
    R *AE0 = P<R>(L.work);
    constexpr int CM_CW = cm_cw_variant(NS);
    const int64_t strips = cm_strips(K, CM_CW), items = cm_items(M, K, N);
    // output products of the item's rows (N <= SKINNY_MAX_N), per wavefront:
    // added at the end of the item, all rows' atomics in flight together
    constexpr int NSX = NS > 0 ? NS : 1;
    static_assert(CM_RB <= 64, "one lane per row of an item");
    __shared__ R zsh[WAVES * CM_RB * 2 * NSX];
    R *zrow = zsh + (threadIdx.x >> 6) * (CM_RB * 2 * NSX);
    const int64_t wave_id = (blockIdx.x * (int64_t)TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * TPB) >> 6;
    for (int64_t it = wave_id; it < items; it += nwaves) {
        const int64_t rb = it / strips, sg = it - rb * strips;
        const int64_t m0 = rb * CM_RB, m1 = m0 + CM_RB < M ? m0 + CM_RB : M;
        const int64_t kb = sg * (64 * CM_CW) + lane;
        R ce[CM_CW], ca0[CM_CW], ca1[CM_CW];
#pragma unroll
        for (int c = 0; c < CM_CW; c++) ce[c] = ca0[c] = ca1[c] = Ring<R>::zero();
        for (int64_t m = m0; m < m1; m++) {
            const uint64_t xm = Ring<R>::mod_s(sdraw(kchi, (uint64_t)m));
            R z0[NS > 0 ? NS : 1], z1[NS > 0 ? NS : 1];
#pragma unroll
            for (int j = 0; j < (NS > 0 ? NS : 1); j++) z0[j] = z1[j] = Ring<R>::zero();
#pragma unroll
            for (int c = 0; c < CM_CW; c++) {
                const int64_t k = kb + 64 * c;
                if (k < K) {
                    const int64_t e = m * K + k;
                    // loads first, streamed (see row_pass_body)
                    const R a0 = ld_nt(P<R>(L.A[0]), e);
                    const R a1 = NS > 0 ? ld_nt(P<R>(L.A[1]), e) : ld(P<R>(L.A[1]), e);
                    const R x0 = ld_nt(P<R>(L.X[0]), e), x1 = ld_nt(P<R>(L.X[1]), e);
                    const R ta0 = ld_nt(P<R>(L.tA[0]), e), ta1 = ld_nt(P<R>(L.tA[1]), e);
                    R tx0 = Ring<R>::zero(), tx1 = Ring<R>::zero();
                    if (check) {
                        tx0 = ld_nt(P<R>(L.tX[0]), e);
                        tx1 = ld_nt(P<R>(L.tX[1]), e);
                    }
                    const R E = add(sub(x0, a0), sub(x1, a1));
                    st(P<R>(L.E), e, E);
                    if (check) {
                        const uint64_t x = Ring<R>::mod_s(sdraw(kce, (uint64_t)e));
                        chk[0] = mad64(chk[0], sub(tx0, ta0), x);
                        chk[1] = mad64(chk[1], sub(tx1, ta1), x);
                        chk[2] = mad64(chk[2], E, x);
                    }
                    ce[c] = mad64(ce[c], E, xm);
                    ca0[c] = mad64(ca0[c], ta0, xm);
                    ca1[c] = mad64(ca1[c], ta1, xm);
                    if constexpr (NS == 0) {
                        st(AE0, e, add(a0, E));  // folded left operand of party 0's product
                    } else {
#pragma unroll
                        for (int j = 0; j < NS; j++) {
                            if (j < N) {
                                const int64_t kn = k * N + j;
                                const R u = ld(P<R>(L.U), kn);
                                z0[j] = mad(mad(z0[j], E, add(ld(P<R>(L.B[0]), kn), u)), a0, u);
                                z1[j] = mad(mad(z1[j], E, ld(P<R>(L.B[1]), kn)), a1, u);
                            }
                        }
                    }
                }
            }
            if constexpr (NS > 0) {
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    if (j < N) {
                        z0[j] = wave_sum(z0[j]);
                        z1[j] = wave_sum(z1[j]);
                        if (lane == 0) {
                            zrow[(m - m0) * 2 * NSX + 2 * j] = z0[j];
                            zrow[(m - m0) * 2 * NSX + 2 * j + 1] = z1[j];
                        }
                    }
                }
            }
        }
        if constexpr (NS > 0) {
            // lane r adds row m0 + r's products (written to LDS by lane 0 of
            // this wavefront)
            wave_sync();
            const int64_t m = m0 + lane;
            if (m < m1) {
                R *cell[2 * NS];
                R val[2 * NS];
                bool ok[2 * NS];
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    cell[2 * j] = P<R>(L.Z[0]) + m * N + j;
                    cell[2 * j + 1] = P<R>(L.Z[1]) + m * N + j;
                    val[2 * j] = zrow[lane * 2 * NSX + 2 * j];
                    val[2 * j + 1] = zrow[lane * 2 * NSX + 2 * j + 1];
                    ok[2 * j] = ok[2 * j + 1] = j < N;
                }
                atomic_add128_n<2 * NS>(cell, val, ok);
            }
        }
#pragma unroll
        for (int c = 0; c < CM_CW; c++) {
            const int64_t k = kb + 64 * c;
            if (k < K) add_cells<3>(P<R>(L.cvec), {o.Uc, o.tBc0, o.tBc1}, k, {ce[c], ca0[c], ca1[c]});
        }
    }
}

// Layers compressed along M (CompactTag only) take k_row_pass_cm, every
// other layer k_row_pass; each returns at once for the layers of the other.
template <class R, int NS>
__global__ __launch_bounds__(TPB) void k_row_pass(const LayerDev *__restrict__ Ls, int flags) {
    const LayerDev &L = Ls[blockIdx.y];
    if (row_variant(L.N) != NS || ((flags & F_COMPACT) && L.cm)) return;
    R chk[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    row_pass_body<R, NS>(L, flags, chk, hw_grid());
    if (flags & F_CHECK)
        wave_accumulate_limbs<3>(chk, rp_cells<R>(L) + 12 * (((blockIdx.x * TPB + threadIdx.x) >> 6) % RP_COPIES));
}

// Three workgroups per compute unit (at most 168 registers) for the 128-bit
// single-output variant, the classifier's: the pass is bound by HBM and a
// third wavefront per SIMD keeps more loads in flight.
template <class R, int NS>
__global__ __launch_bounds__(TPB, (sizeof(R) == 16 && NS == 1) ? 3 : 1) void k_row_pass_cm(
    const LayerDev *__restrict__ Ls, int flags) {
    const LayerDev &L = Ls[blockIdx.y];
    if (row_variant(L.N) != NS || !L.cm) return;
    R chk[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    row_pass_cm<R, NS>(L, flags, chk);
    if (flags & F_CHECK)
        wave_accumulate_limbs<3>(chk, rp_cells<R>(L) + 12 * (((blockIdx.x * TPB + threadIdx.x) >> 6) % RP_COPIES));
}

template <class R>
void launch_row_variants(const dim3 &g, const LayerDev *L, int flags, int variants, hipStream_t st) {
    const dim3 b(TPB);
    if (variants & (1 << 0)) hipLaunchKernelGGL((k_row_pass<R, 0>), g, b, 0, st, L, flags);
    if (variants & (1 << 1)) hipLaunchKernelGGL((k_row_pass<R, 1>), g, b, 0, st, L, flags);
    if (variants & (1 << 2)) hipLaunchKernelGGL((k_row_pass<R, 2>), g, b, 0, st, L, flags);
    if (variants & (1 << 4)) hipLaunchKernelGGL((k_row_pass<R, 4>), g, b, 0, st, L, flags);
    if (variants & (1 << 8)) hipLaunchKernelGGL((k_row_pass<R, SKINNY_MAX_N>), g, b, 0, st, L, flags);
    if (variants & (1 << (VARIANT_CM + 0))) hipLaunchKernelGGL((k_row_pass_cm<R, 0>), g, b, 0, st, L, flags);
    if (variants & (1 << (VARIANT_CM + 1))) hipLaunchKernelGGL((k_row_pass_cm<R, 1>), g, b, 0, st, L, flags);
    if (variants & (1 << (VARIANT_CM + 2))) hipLaunchKernelGGL((k_row_pass_cm<R, 2>), g, b, 0, st, L, flags);
    if (variants & (1 << (VARIANT_CM + 4))) hipLaunchKernelGGL((k_row_pass_cm<R, 4>), g, b, 0, st, L, flags);
    if (variants & (1 << (VARIANT_CM + 8))) hipLaunchKernelGGL((k_row_pass_cm<R, SKINNY_MAX_N>), g, b, 0, st, L, flags);
}

hipError_t launch_row_pass(int eb, const LayerDev *L, int n, int flags, int64_t max_items, int variants, hipStream_t st) {
    // at most 8192 workgroups, each sweeping many items: every workgroup adds
    // its check sums into one of RP_COPIES copies without waiting
    const int gx = grid_items(max_items);
    const dim3 g(gx > 8192 ? 8192 : gx, n);
    if (eb == 8) launch_row_variants<r64>(g, L, flags, variants, st);
    else launch_row_variants<u128>(g, L, flags, variants, st);
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
// [tZ^f]_p = [tR^f]_p - [Delta]_p (D mod 2^64) / 2^f.  (post_body, ct_passes.h)

template <class R>
__global__ __launch_bounds__(TPB) void k_post(const LayerDev *__restrict__ Ls, int flags) {
    post_body<R>(Ls, flags, hw_grid());
}

hipError_t launch_post(int eb, const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st) {
    LAUNCH_RING(eb, k_post, dim3(grid_items(max_items), n), dim3(TPB), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- compact tag
// Products of the compact tag of a layer compressed along M, over K x N
// (Eq. (5) multiplied by chi^T from the left), per column n:
//   (E^c U)_n = sum_k E^c_k U_kn,
//   [tZ^c]_p,n partial = sum_k (E^c_k [tB]_p,kn + [tA^c]_p,k U_kn);
// k_compact_final adds [tC^c]_p and [Delta]_p (E^c U).
template <class R>
__global__ __launch_bounds__(TPB) void k_col_tag(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y];
    if (!L.cm) return;
    const int64_t N = L.N;
    const CvecOff o = cvec_off(N, L.K);
    R *cv = P<R>(L.cvec);
    auto elem = [&](int64_t k, int64_t n, R (&v)[3]) {
        const int64_t e = kn_src(L.cv, N, k, n);  // a convolution's implicit im2col entry
        if (e < 0) return;
        const R ec = ld(cv + o.Uc, k), u = ld(P<R>(L.U), e);
        v[0] = mad(v[0], ec, u);
        v[1] = mad(mad(v[1], ec, ld(P<R>(L.tB[0]), e)), ld(cv + o.tBc0, k), u);
        v[2] = mad(mad(v[2], ec, ld(P<R>(L.tB[1]), e)), ld(cv + o.tBc1, k), u);
    };
    auto done = [&](int64_t n, R (&v)[3]) { add_cells<3>(cv, {o.EUc, o.tZc0, o.tZc1}, n, v); };
    col_sweep<R, 3>(hw_grid(), L.K, N, elem, done);
}

hipError_t launch_col_tag(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st) {
    LAUNCH_RING(eb, k_col_tag, dim3(grid_items(max_items), n), dim3(TPB), st, L);
    return hipGetLastError();
}

// Eq. (5) with the key on the public term, per entry i of the compressed
// vectors (a row m; for a layer compressed along M, a column n):
//   [tZ^c]_p = [tC^c]_p + (E [tB^c]_p + [tA]_p U^c) + [Delta]_p (E U^c),
//   [tD^c]_p = [tR^c]_p - [tZ^c]_p.
// F_CHECK: the compact check of D (Fig. 7 verification steps 2-5) in the
// accumulator form of the batch checks,
//   acc6 = -sum chihat_i [tD^c]_{0,i}, acc7 = -sum chihat_i [tD^c]_{1,i},
//   acc8 = -sum chihat_i D^c_i,  so cs_p = acc_{6+p} - [Delta]_p acc8
//        = sum_i chihat_i ([Delta]_p D^c_i - [tD^c]_{p,i})   (mod 2^128).
template <class R>
__global__ __launch_bounds__(TPB) void k_compact_final(const LayerDev *__restrict__ Ls, int flags) {
    compact_final_body<R>(Ls, flags, hw_grid());
}

hipError_t launch_compact_final(int eb, const LayerDev *L, int n, int flags, hipStream_t st) {
    LAUNCH_RING(eb, k_compact_final, dim3(4, n), dim3(TPB), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- MAC checks
// Standalone verification (ct_mac_check): Pi_BatchRec tag check (Fig. 1) of
// an opened W = P - Q with one public combiner chi'_e per element (drawn from
// the layer's stream; never stored):
//   acc0 = sum chi' ([tP]_0 - [tQ]_0),  acc1 = sum chi' ([tP]_1 - [tQ]_1),
//   accW = sum chi' W;   cs_p = acc_p - [Delta]_p accW   (mod 2^128).
// y = layer * 3 + which; which = 0: E (X, A), 1: U (Y, B), 2: D (R, Z).
template <class R>
__global__ __launch_bounds__(TPB) void k_check_batch(const LayerDev *__restrict__ Ls, int which_mask) {
    __shared__ R sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y / 3];
    const int which = blockIdx.y % 3;
    if (!((which_mask >> which) & 1)) return;
    int64_t n;
    const R *tP0, *tP1, *tQ0, *tQ1, *W;
    uint64_t key;
    if (which == 0) {
        n = L.M * L.K; tP0 = P<R>(L.tX[0]); tP1 = P<R>(L.tX[1]); tQ0 = P<R>(L.tA[0]); tQ1 = P<R>(L.tA[1]); W = P<R>(L.E); key = L.key[K_CHI_E];
    } else if (which == 1) {
        n = L.nr; tP0 = P<R>(L.tY[0]); tP1 = P<R>(L.tY[1]); tQ0 = P<R>(L.tB[0]); tQ1 = P<R>(L.tB[1]); W = P<R>(L.U); key = L.key[K_CHI_U];
    } else {
        n = L.M * L.N; tP0 = P<R>(L.tR[0]); tP1 = P<R>(L.tR[1]); tQ0 = P<R>(L.tZ[0]); tQ1 = P<R>(L.tZ[1]); W = P<R>(L.D); key = L.key[K_CHI_D];
    }
    if (blockIdx.x * (int64_t)TPB >= n) return;  // no elements for this workgroup
    R v[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const uint64_t c = Ring<R>::mod_s(sdraw(key, (uint64_t)e));
        v[0] = mad64(v[0], sub(ld(tP0, e), ld(tQ0, e)), c);
        v[1] = mad64(v[1], sub(ld(tP1, e), ld(tQ1, e)), c);
        v[2] = mad64(v[2], ld(W, e), c);
    }
    block_accumulate<3>(v, sh, P<R>(L.acc) + 3 * which);
}

hipError_t launch_check_batch(int eb, const LayerDev *L, int n, int which_mask, int64_t max_elems, hipStream_t st) {
    int g = grid_for(max_elems);
    if (g > 2048) g = 2048;
    LAUNCH_RING(eb, k_check_batch, dim3(g, 3 * n), dim3(TPB), st, L, which_mask);
    return hipGetLastError();
}

// Standalone compact check of D from the stored compact vectors (same
// accumulator form as in k_compact_final).
template <class R>
__global__ __launch_bounds__(TPB) void k_check_compact(const LayerDev *__restrict__ Ls) {
    __shared__ R sh[3 * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t M = cvec_rows(L);
    const CvecOff o = cvec_off(M, L.K);
    R v[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    for (int64_t i = threadIdx.x; i < M; i += TPB) {
        const uint64_t c = Ring<R>::mod_s(sdraw(L.key[K_CHIHAT], (uint64_t)i));
        v[0] = mad64(v[0], ld(P<R>(L.cvec) + o.tDc0, i), c);
        v[1] = mad64(v[1], ld(P<R>(L.cvec) + o.tDc1, i), c);
        v[2] = mad64(v[2], ld(P<R>(L.cvec) + o.Dc, i), c);
    }
    block_sum<3, WAVES>(v, sh);
    if (threadIdx.x == 0) {
        st(P<R>(L.acc), 6, sub(Ring<R>::zero(), v[0]));
        st(P<R>(L.acc), 7, sub(Ring<R>::zero(), v[1]));
        st(P<R>(L.acc), 8, sub(Ring<R>::zero(), v[2]));
    }
}

hipError_t launch_check_compact(int eb, const LayerDev *L, int n, hipStream_t st) {
    LAUNCH_RING(eb, k_check_compact, dim3(1, n), dim3(TPB), st, L);
    return hipGetLastError();
}

// cs[W][p] = acc[3W + p] - [Delta]_p acc[3W + 2]; accept iff every cs sum is 0
// (finalize_body, one wavefront per layer).
template <class R>
__global__ __launch_bounds__(64) void k_finalize(const LayerDev *__restrict__ Ls, int n, ct_check_result *out) {
    finalize_body<R>(Ls, n, out, blockIdx.x);
}

hipError_t launch_finalize(int eb, const LayerDev *L, int n, ct_check_result *out, hipStream_t st) {
    LAUNCH_RING(eb, k_finalize, dim3(n), dim3(64), st, L, n, out);
    return hipGetLastError();
}

}  // namespace ct
