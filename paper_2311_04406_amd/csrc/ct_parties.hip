// ct_parties.hip -- the linear-layer path for more than two parties (the
// paper's appendix on scaling with parties): n = 3 .. CT_MAX_PARTIES parties
// simulated in one process, every per-party step of the two-party path done
// for each party, every opening a sum over all parties' broadcasts.
//
// They share the matrix-core products (k_pack, k_ring_gemm: one product per
// party) with the two-party path:
//   dealer   k_np_lift, k_np_auth: n-way authenticated sharing (Sec. 2.4);
//   online   k_np_row_pass, the fused pass over M x K of matrix-core layers
//            and layers with N <= 2 (E, its check sums, the folded operands,
//            the compact-tag row products and, for N <= 2, the output
//            products of every party); k_np_open_e for the other layers and
//            k_np_open_u (Fig. 7 step 1); the products (Eq. (2), and Eq. (3)
//            in SPDZ2k mode) on the matrix cores or, for 2 < N <=
//            SKINNY_MAX_N, in k_np_skinny; k_np_post (D, Pi_OptMAC,
//            truncation), k_np_compress, k_np_gemv, k_np_compact_final
//            (Fig. 7 steps 5-7, Eq. (5));
//   checks   accumulated by the passes (F_CHECK) or by k_np_check_batch /
//            k_np_check_compact, then k_np_finalize.
// Check accumulators of a layer: acc[W ACC_W + p] = sum chi [tW]_p for p < n,
// acc[W ACC_W + MAXP] = sum chi W, W in (E, U, D); the fused row pass adds
// its E sums into NP_RP_COPIES limb-celled copies instead (ct_internal.h).
#include <algorithm>

#include "ct_sweep.h"

namespace ct {

template <class R>
__device__ __forceinline__ R key_sum_np(const LayerDev &L) {
    R r;
    key_sum_np_to(L, r);
    return r;
}

// ---------------------------------------------------------------- dealer
// The lifts A~ (M x K) and B~ (K x N) go to the last party's buffers; the
// triple product C~ = A~ B~ is formed there by the matrix cores (or
// k_skinny), and k_np_auth splits every lift into the parties' shares.
template <class R>
__global__ void k_np_lift(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y >> 1];
    const int which = blockIdx.y & 1, last = L.np - 1;
    const int64_t n = which ? L.K * L.N : L.M * L.K;
    const uint64_t key = which ? L.key[K_LIFT_B] : L.key[K_LIFT_A];
    R *dst = which ? P<R>(L.B[last]) : P<R>(L.A[last]);
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB)
        st(dst, e, Ring<R>::draw(key, (uint64_t)e));
}

hipError_t launch_np_lift(int eb, const LayerDev *L, int n, int64_t max_elems, hipStream_t st) {
    LAUNCH_RING(eb, k_np_lift, dim3(grid_for(max_elems), 2 * n), dim3(TPB), st, L);
    return hipGetLastError();
}

// n-way authenticated sharing of every lifted value: parties 0 .. n-2 draw
// their value and tag shares (party p from the streams of purpose 0x10 / 0x20
// + object + 256 p), the last party completes sum_p [v]_p = v~ and
// sum_p [t]_p = Delta~ v~ with Delta~ the sum of the n key shares.
template <class R>
__global__ void k_np_auth(const LayerDev *__restrict__ Ls, int obj_mask) {
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
    const int last = L.np - 1;
    const R dsum = key_sum_np<R>(L);
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        R lift;
        if (obj == OBJ_X) lift = Ring<R>::input(sdraw(L.key[K_LIFT_X], (uint64_t)e), L.in_bits);
        else if (obj == OBJ_Y) lift = Ring<R>::input(sdraw(L.key[K_LIFT_Y], (uint64_t)e), L.in_bits);
        else if (obj == OBJ_R) lift = Ring<R>::draw(L.key[K_LIFT_R], (uint64_t)e);
        else if (obj == OBJ_RF)
            lift = Ring<R>::lift(Ring<R>::mod_k(Ring<R>::draw(L.key[K_LIFT_R], (uint64_t)e)) >> L.f,
                                 Ring<R>::mod_s(sdraw(L.key[K_LIFT_RF], (uint64_t)e)));
        else lift = ld(P<R>(v[last]), e);  // A~, B~ or C~ in the last party's buffer
        R sv = Ring<R>::zero(), stg = Ring<R>::zero();
        for (int p = 0; p < last; p++) {
            const uint64_t kv = p == 0 ? L.key[K_VSH_X + obj - 1] : L.vsh[p - 1][obj - 1];
            const uint64_t kt = p == 0 ? L.key[K_TSH_X + obj - 1] : L.tsh[p - 1][obj - 1];
            const R a = Ring<R>::draw(kv, (uint64_t)e), b = Ring<R>::draw(kt, (uint64_t)e);
            st(P<R>(v[p]), e, a);
            st(P<R>(t[p]), e, b);
            sv = add(sv, a);
            stg = add(stg, b);
        }
        st(P<R>(v[last]), e, sub(lift, sv));
        st(P<R>(t[last]), e, sub(mul(lift, dsum), stg));
    }
}

hipError_t launch_np_auth(int eb, const LayerDev *L, int n, int obj_mask, int64_t max_elems, hipStream_t st) {
    LAUNCH_RING(eb, k_np_auth, dim3(grid_for(max_elems), NUM_OBJ * n), dim3(TPB), st, L, obj_mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------- zeroing
// what bit 0: the compact vectors ((1 + n) K + (2 + 4 n) M elements); bit 1:
// the check accumulators; bit 2: for layers with N <= 2, [Z]_p = [C]_p (the
// fused row pass adds their row products atomically); bit 3: also
// [tZ]_p = [tC]_p.
template <class R>
__global__ void k_np_zero(const LayerDev *__restrict__ Ls, int what) {
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t t0 = blockIdx.x * (int64_t)TPB + threadIdx.x, stride = (int64_t)gridDim.x * TPB;
    if (what & 1) {
        const int64_t n = (1 + L.np) * L.K + (2 + 4 * L.np) * L.M;
        for (int64_t e = t0; e < n; e += stride) st(P<R>(L.cvec), e, Ring<R>::zero());
    }
    if ((what & 2) && blockIdx.x == 0)  // ACC_PER_LAYER 16-byte elements whatever the ring
        for (int i = threadIdx.x; i < ACC_PER_LAYER; i += TPB) st(L.acc, i, u128{0, 0});
    if ((what & 4) && L.N <= 2) {
        const int64_t n = L.M * L.N;
        for (int64_t e = t0; e < n; e += stride)
            for (int p = 0; p < L.np; p++) {
                st(P<R>(L.Z[p]), e, ld(P<R>(L.C[p]), e));
                if (what & 8) st(P<R>(L.tZ[p]), e, ld(P<R>(L.tC[p]), e));
            }
    }
}

hipError_t launch_np_zero(int eb, const LayerDev *L, int n, int what, int64_t max_elems, hipStream_t st) {
    LAUNCH_RING(eb, k_np_zero, dim3((what & 5) ? grid_for(max_elems) : 1, n), dim3(TPB), st, L, what);
    return hipGetLastError();
}

// ---------------------------------------------------------------- openings
// E = sum_p ([X]_p - [A]_p) (Fig. 7 step 1).  For matrix-core layers also the
// folded left operands A_0 + E and, in SPDZ2k mode, [tA]_p + [Delta]_p E
// (workspace, M K elements each).  F_CHECK: the batch check sums of E.
template <class R>
__global__ __launch_bounds__(TPB) void k_np_open_e(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ R sh[ACC_W * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    if (np_fused_row(L.N)) return;  // opened by k_np_row_pass
    const int np = L.np;
    const bool check = flags & F_CHECK, spdz = flags & F_SPDZ, wide = L.N > SKINNY_MAX_N;
    const int64_t n = L.M * L.K;
    R *W = P<R>(L.work);
    R chk[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) chk[i] = Ring<R>::zero();
    const uint64_t kce = L.key[K_CHI_E];
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        R E = Ring<R>::zero();
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) E = add(E, sub(ld(P<R>(L.X[p]), e), ld(P<R>(L.A[p]), e)));
        st(P<R>(L.E), e, E);
        if (wide) {
            st(W, e, add(ld(P<R>(L.A[0]), e), E));
            if (spdz) {
#pragma unroll
                for (int p = 0; p < MAXP; p++)
                    if (p < np) st(W + (1 + p) * n, e, add(ld(P<R>(L.tA[p]), e), mul64(E, L.delta[p])));
            }
        }
        if (check) {
            const uint64_t x = Ring<R>::mod_s(sdraw(kce, (uint64_t)e));
#pragma unroll
            for (int p = 0; p < MAXP; p++)
                if (p < np) chk[p] = mad64(chk[p], sub(ld(P<R>(L.tX[p]), e), ld(P<R>(L.tA[p]), e)), x);
            chk[MAXP] = mad64(chk[MAXP], E, x);
        }
    }
    if (check) block_accumulate<ACC_W>(chk, sh, P<R>(L.acc) + 0 * ACC_W);
}

// U = sum_p ([Y]_p - [B]_p); F_CHECK: the batch check sums of U.
template <class R>
__global__ __launch_bounds__(TPB) void k_np_open_u(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ R sh[ACC_W * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int np = L.np;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT;
    const int64_t N = L.N;
    R chk[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) chk[i] = Ring<R>::zero();
    const uint64_t kcu = L.key[K_CHI_U], kchi = L.key[K_CHI];
    const NpCvec o = np_cvec(L.M, L.K, np);
    R *cv = P<R>(L.cvec);
    // a sweep over the rows of K x N, so that CompactTag's compressions along
    // N, U^c = U chi and [tB^c]_p = [tB]_p chi, are formed from the values
    // this pass has in registers (no second read of U and [tB]_p)
    auto elem = [&](int64_t r, int64_t c, R (&v)[1 + MAXP]) {
        const int64_t e = r * N + c;
        R U = Ring<R>::zero(), tb[MAXP];
#pragma unroll
        for (int p = 0; p < MAXP; p++) {
            tb[p] = Ring<R>::zero();
            if (p < np) {
                U = add(U, sub(ld_nt(P<R>(L.Y[p]), e), ld(P<R>(L.B[p]), e)));
                if (check || compact) tb[p] = ld_nt(P<R>(L.tB[p]), e);
            }
        }
        st(P<R>(L.U), e, U);
        if (check) {
            const uint64_t x = Ring<R>::mod_s(sdraw(kcu, (uint64_t)e));
#pragma unroll
            for (int p = 0; p < MAXP; p++)
                if (p < np) chk[p] = mad64(chk[p], sub(ld_nt(P<R>(L.tY[p]), e), tb[p]), x);
            chk[MAXP] = mad64(chk[MAXP], U, x);
        }
        if (compact) {
            const uint64_t x = Ring<R>::mod_s(sdraw(kchi, (uint64_t)c));
            v[0] = mad64(v[0], U, x);
#pragma unroll
            for (int p = 0; p < MAXP; p++) if (p < np) v[1 + p] = mad64(v[1 + p], tb[p], x);
        }
    };
    auto done = [&](int64_t r, R (&v)[1 + MAXP]) {
        if (!compact) return;
        atomic_add128(cv + o.Uc + r, v[0]);
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) atomic_add128(cv + o.tb(p) + r, v[1 + p]);
    };
    row_sweep<R, 1 + MAXP>(hw_grid(), L.K, N, elem, done);
    if (check) block_accumulate<ACC_W>(chk, sh, P<R>(L.acc) + 1 * ACC_W);
}

// which: bit 0 opens E (layers the fused row pass does not serve), bit 1 opens U.
// The elementwise passes that accumulate check sums run at most 1024
// workgroups per layer: each adds its sums with one atomic per accumulator,
// and same-address atomics serialize.
inline int grid_acc(int64_t n) { return std::min(grid_for(n), 1024); }

hipError_t launch_np_open(int eb, const LayerDev *L, int n, int which, int flags, int64_t max_elems, hipStream_t st) {
    if (which & 1) LAUNCH_RING(eb, k_np_open_e, dim3(grid_acc(max_elems), n), dim3(TPB), st, L, flags);
    if (which & 2) LAUNCH_RING(eb, k_np_open_u, dim3(grid_acc(max_elems), n), dim3(TPB), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fused row pass
// One pass over M x K for matrix-core layers and layers with N <= 2 (the
// n-party form of the two-party row pass): opens E = sum_p ([X]_p - [A]_p),
// accumulates its batch check sums, writes the folded left operands
// (A_0 + E; SPDZ2k [tA]_p + [Delta]_p E), adds the row products of the compact
// tag (E U^c and per party E [tB^c]_p + [tA]_p U^c, onto zeroed vectors) and,
// for N <= 2, forms every party's output row products
//   [Z]_p = [C]_p + E [B]_p + L_p U (L_0 = A_0 + E, L_p = [A]_p),
//   [tZ]_p = [tC]_p + E [tB]_p + ([tA]_p + [Delta]_p E) U (SPDZ2k),
// added onto [Z]_p = [C]_p ([tZ]_p = [tC]_p) set by k_np_zero.  Items are row
// segments of row_seg(M, K) elements taken segment-major, one wavefront each.
// NP: the party count, a compile-time constant so that only NP parties'
// accumulators take registers.
template <class R, int NS, int NP>
__global__ __launch_bounds__(TPB) void k_np_row_pass(const LayerDev *__restrict__ Ls, int flags) {
    const LayerDev &L = Ls[blockIdx.y];
    if (!np_fused_row(L.N) || row_variant(L.N) != NS || L.np != NP) return;
    constexpr int NZ = NS > 0 ? NS : 1;
    constexpr int np = NP;
    const int lane = threadIdx.x & 63;
    const int64_t M = L.M, K = L.K, N = L.N, mk = M * K;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT, spdz = flags & F_SPDZ;
    const NpCvec o = np_cvec(M, K, np);
    R *cv = P<R>(L.cvec);
    R *W = P<R>(L.work);
    const uint64_t kce = L.key[K_CHI_E];
    R chk[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) chk[i] = Ring<R>::zero();
    const int64_t seg = row_seg(M, K), items = M * ((K + seg - 1) / seg);
    const int64_t wave_id = (blockIdx.x * (int64_t)TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * TPB) >> 6;
    for (int64_t it = wave_id; it < items; it += nwaves) {
        const int64_t sg = it / M, m = it - sg * M, k0 = sg * seg;
        const int64_t k1 = k0 + seg < K ? k0 + seg : K;
        R cp[1 + MAXP];  // E U^c, then per party E [tB^c]_p + [tA]_p U^c
#pragma unroll
        for (int i = 0; i < 1 + MAXP; i++) cp[i] = Ring<R>::zero();
        R z[MAXP][NZ], t[MAXP][NZ];
#pragma unroll
        for (int p = 0; p < MAXP; p++)
#pragma unroll
            for (int j = 0; j < NZ; j++) z[p][j] = t[p][j] = Ring<R>::zero();
        const bool need_ta = check || compact || spdz;
        for (int64_t k = k0 + lane; k < k1; k += 64) {
            const int64_t e = m * K + k;
            // every load of the element is issued before the store of E (which
            // the compiler may not move loads across); the arrays are
            // streamed, except [A]_p (p > 0) of a matrix-core layer, which
            // k_pack reads next
            R a[MAXP], x[MAXP], ta[MAXP], tx[MAXP];
#pragma unroll
            for (int p = 0; p < MAXP; p++) {
                a[p] = x[p] = ta[p] = tx[p] = Ring<R>::zero();
                if (p < np) {
                    a[p] = (NS > 0 || p == 0) ? ld_nt(P<R>(L.A[p]), e) : ld(P<R>(L.A[p]), e);
                    x[p] = ld_nt(P<R>(L.X[p]), e);
                    if (need_ta) ta[p] = ld_nt(P<R>(L.tA[p]), e);
                    if (check) tx[p] = ld_nt(P<R>(L.tX[p]), e);
                }
            }
            R E = Ring<R>::zero();
#pragma unroll
            for (int p = 0; p < MAXP; p++)
                if (p < np) E = add(E, sub(x[p], a[p]));
            // E of a layer whose products are formed here is not read again
            // in the step; a matrix-core layer's is packed next
            if constexpr (NS > 0) st_nt(P<R>(L.E), e, E);
            else st(P<R>(L.E), e, E);
            if constexpr (NS == 0) {
                st(W, e, add(a[0], E));
            }
            uint64_t xe = 0;
            if (check) {
                xe = Ring<R>::mod_s(sdraw(kce, (uint64_t)e));
                chk[MAXP] = mad64(chk[MAXP], E, xe);
            }
            const R uc = compact ? ld(cv + o.Uc, k) : Ring<R>::zero();
            if (compact) cp[0] = mad(cp[0], E, uc);
#pragma unroll
            for (int p = 0; p < MAXP; p++) {
                if (p < np) {
                    if (check) chk[p] = mad64(chk[p], sub(tx[p], ta[p]), xe);
                    if (compact) cp[1 + p] = mad(mad(cp[1 + p], E, ld(cv + o.tb(p), k)), ta[p], uc);
                    const R tae = spdz ? add(ta[p], mul64(E, L.delta[p])) : Ring<R>::zero();
                    if constexpr (NS == 0) {
                        if (spdz) st(W + (1 + p) * mk, e, tae);  // folded tag operand of party p
                    } else {
                        const R ap = p == 0 ? add(a[0], E) : a[p];
#pragma unroll
                        for (int j = 0; j < NS; j++) {
                            if (j < N) {
                                const int64_t kn = k * N + j;
                                const R u = ld(P<R>(L.U), kn);
                                z[p][j] = mad(mad(z[p][j], E, ld(P<R>(L.B[p]), kn)), ap, u);
                                if (spdz) t[p][j] = mad(mad(t[p][j], E, ld(P<R>(L.tB[p]), kn)), tae, u);
                            }
                        }
                    }
                }
            }
        }
        if (compact) {
#pragma unroll
            for (int i = 0; i < 1 + MAXP; i++)
                if (i < 1 + np) cp[i] = wave_sum(cp[i]);
            if (lane == 0) {
                atomic_add128(cv + o.EUc + m, cp[0]);
#pragma unroll
                for (int p = 0; p < MAXP; p++)
                    if (p < np) atomic_add128(cv + o.tz(p) + m, cp[1 + p]);
            }
        }
        if constexpr (NS > 0) {
#pragma unroll
            for (int p = 0; p < MAXP; p++) {
                if (p < np) {
#pragma unroll
                    for (int j = 0; j < NS; j++) {
                        if (j < N) {
                            z[p][j] = wave_sum(z[p][j]);
                            if (spdz) t[p][j] = wave_sum(t[p][j]);
                            if (lane == 0) {
                                atomic_add128(P<R>(L.Z[p]) + m * N + j, z[p][j]);
                                if (spdz) atomic_add128(P<R>(L.tZ[p]) + m * N + j, t[p][j]);
                            }
                        }
                    }
                }
            }
        }
    }
    if (check)
        wave_accumulate_limbs<ACC_W>(chk, rp_cells<R>(L) + 4 * ACC_W * (((blockIdx.x * TPB + threadIdx.x) >> 6) % NP_RP_COPIES));
}

template <class R, int NP>
void launch_np_row_variants(const dim3 &g, const LayerDev *L, int flags, int variants, hipStream_t st) {
    const dim3 b(TPB);
    if (variants & (1 << 0)) hipLaunchKernelGGL((k_np_row_pass<R, 0, NP>), g, b, 0, st, L, flags);
    if (variants & (1 << 1)) hipLaunchKernelGGL((k_np_row_pass<R, 1, NP>), g, b, 0, st, L, flags);
    if (variants & (1 << 2)) hipLaunchKernelGGL((k_np_row_pass<R, 2, NP>), g, b, 0, st, L, flags);
}

template <class R>
void launch_np_row_parties(int np, const dim3 &g, const LayerDev *L, int flags, int variants, hipStream_t st) {
    static_assert(MAXP == 5, "one instantiation per party count");
    if (np == 3) launch_np_row_variants<R, 3>(g, L, flags, variants, st);
    else if (np == 4) launch_np_row_variants<R, 4>(g, L, flags, variants, st);
    else launch_np_row_variants<R, 5>(g, L, flags, variants, st);
}

hipError_t launch_np_row_pass(int eb, int np, const LayerDev *L, int n, int flags, int64_t max_items, int variants,
                              hipStream_t st) {
    // at most 8192 workgroups: each adds its check sums into one of
    // NP_RP_COPIES copies without waiting
    const dim3 g(std::min(grid_items(max_items), 8192), n);
    if (eb == 8) launch_np_row_parties<r64>(np, g, L, flags, variants, st);
    else launch_np_row_parties<u128>(np, g, L, flags, variants, st);
    return hipGetLastError();
}

// Layers with N <= SKINNY_MAX_N: one wavefront per (row m, party p) forms
//   [Z]_p = [C]_p + E [B]_p + L_p U,  L_0 = A_0 + E, L_p = [A]_p   (Eq. (2)),
// and in SPDZ2k mode [tZ]_p = [tC]_p + E [tB]_p + ([tA]_p + [Delta]_p E) U (Eq. (3)).
template <class R>
__global__ __launch_bounds__(TPB) void k_np_skinny(const LayerDev *__restrict__ Ls, int flags) {
    const LayerDev &L = Ls[blockIdx.y];
    const int64_t M = L.M, K = L.K, N = L.N;
    if (np_fused_row(N)) return;
    const int np = L.np, lane = threadIdx.x & 63;
    const bool spdz = flags & F_SPDZ;
    const int64_t items = M * np;
    const int64_t wave_id = (blockIdx.x * (int64_t)TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * TPB) >> 6;
    for (int64_t it = wave_id; it < items; it += nwaves) {
        const int64_t m = it / np;
        const int p = (int)(it - m * np);
        R z[SKINNY_MAX_N], t[SKINNY_MAX_N];
#pragma unroll
        for (int j = 0; j < SKINNY_MAX_N; j++) z[j] = t[j] = Ring<R>::zero();
        for (int64_t k = lane; k < K; k += 64) {
            const int64_t e = m * K + k;
            const R E = ld(P<R>(L.E), e);
            R a = ld(P<R>(L.A[p]), e);
            if (p == 0) a = add(a, E);
            const R ta = spdz ? add(ld(P<R>(L.tA[p]), e), mul64(E, L.delta[p])) : Ring<R>::zero();
#pragma unroll
            for (int j = 0; j < SKINNY_MAX_N; j++) {
                if (j < N) {
                    const int64_t kn = k * N + j;
                    const R u = ld(P<R>(L.U), kn);
                    z[j] = mad(mad(z[j], E, ld(P<R>(L.B[p]), kn)), a, u);
                    if (spdz) t[j] = mad(mad(t[j], E, ld(P<R>(L.tB[p]), kn)), ta, u);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < SKINNY_MAX_N; j++) {
            if (j < N) {
                z[j] = wave_sum(z[j]);
                if (spdz) t[j] = wave_sum(t[j]);
                if (lane == 0) {
                    const int64_t mn = m * N + j;
                    st(P<R>(L.Z[p]), mn, add(ld(P<R>(L.C[p]), mn), z[j]));
                    if (spdz) st(P<R>(L.tZ[p]), mn, add(ld(P<R>(L.tC[p]), mn), t[j]));
                }
            }
        }
    }
}

hipError_t launch_np_skinny(int eb, const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st) {
    LAUNCH_RING(eb, k_np_skinny, dim3(grid_items(max_items), n), dim3(TPB), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pass over M x N
// D = sum_p ([R]_p - [Z]_p); f > 0: [Z^f]_p = [R^f]_p - (D mod 2^k) / 2^f
// (party 0 subtracts the public term), [tZ^f]_p = [tR^f]_p - [Delta]_p (D mod 2^k) / 2^f;
// CompactTag: [tZ]_p = [tR]_p - [Delta]_p D (Pi_OptMAC); SPDZ2k with F_CHECK:
// the batch check sums of D with [tD]_p = [tR]_p - [tZ]_p.
template <class R>
__global__ __launch_bounds__(TPB) void k_np_post(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ R sh[ACC_W * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int np = L.np;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT;
    const int64_t n = L.M * L.N;
    R chk[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) chk[i] = Ring<R>::zero();
    const uint64_t kcd = L.key[K_CHI_D];
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        R D = Ring<R>::zero();
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) D = add(D, sub(ld(P<R>(L.R[p]), e), ld(P<R>(L.Z[p]), e)));
        st(P<R>(L.D), e, D);
        if (L.f > 0) {
            const uint64_t df = Ring<R>::mod_k(D) >> L.f;
#pragma unroll
            for (int p = 0; p < MAXP; p++) if (p < np) {
                const R rf = ld(P<R>(L.Rf[p]), e);
                st(P<R>(L.Zf[p]), e, p == 0 ? sub(rf, Ring<R>::small(df)) : rf);
                st(P<R>(L.tZf[p]), e, sub(ld(P<R>(L.tRf[p]), e), mul64(Ring<R>::small(L.delta[p]), df)));
            }
        }
        if (compact) {
#pragma unroll
            for (int p = 0; p < MAXP; p++)
                if (p < np) st(P<R>(L.tZ[p]), e, sub(ld(P<R>(L.tR[p]), e), mul64(D, L.delta[p])));
        } else if (check) {
            const uint64_t x = Ring<R>::mod_s(sdraw(kcd, (uint64_t)e));
#pragma unroll
            for (int p = 0; p < MAXP; p++)
                if (p < np) chk[p] = mad64(chk[p], sub(ld(P<R>(L.tR[p]), e), ld(P<R>(L.tZ[p]), e)), x);
            chk[MAXP] = mad64(chk[MAXP], D, x);
        }
    }
    if (!compact && check) block_accumulate<ACC_W>(chk, sh, P<R>(L.acc) + 2 * ACC_W);
}

hipError_t launch_np_post(int eb, const LayerDev *L, int n, int flags, int64_t max_elems, hipStream_t st) {
    LAUNCH_RING(eb, k_np_post, dim3(grid_acc(max_elems), n), dim3(TPB), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- compact tag
// Pi_Compress along N (Fig. 7 steps 5-6) of the M x N quantities, chi_c per
// column: D^c, [tR^c]_p, [tC^c]_p (U^c and [tB^c]_p are formed by
// k_np_open_u).
template <class R>
__global__ __launch_bounds__(TPB) void k_np_compress(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y];
    const int np = L.np;
    const NpCvec o = np_cvec(L.M, L.K, np);
    R *cv = P<R>(L.cvec);
    const uint64_t kchi = L.key[K_CHI];
    const int64_t N = L.N;
    auto elem = [&](int64_t r, int64_t c, R (&v)[1 + 2 * MAXP]) {
        const int64_t e = r * N + c;
        const uint64_t x = Ring<R>::mod_s(sdraw(kchi, (uint64_t)c));
        v[0] = mad64(v[0], ld(P<R>(L.D), e), x);
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) {
            v[1 + p] = mad64(v[1 + p], ld(P<R>(L.tR[p]), e), x);
            v[1 + MAXP + p] = mad64(v[1 + MAXP + p], ld(P<R>(L.tC[p]), e), x);
        }
    };
    auto done = [&](int64_t r, R (&v)[1 + 2 * MAXP]) {
        atomic_add128(cv + o.Dc + r, v[0]);
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) {
            atomic_add128(cv + o.tr(p) + r, v[1 + p]);
            atomic_add128(cv + o.tc(p) + r, v[1 + MAXP + p]);
        }
    };
    row_sweep<R, 1 + 2 * MAXP>(hw_grid(), L.M, N, elem, done);
}

hipError_t launch_np_compress(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st) {
    LAUNCH_RING(eb, k_np_compress, dim3(grid_items(max_items), n), dim3(TPB), st, L);
    return hipGetLastError();
}

// Row products of the compact tag over M x K (Eq. (5)): E U^c, and per party
// E [tB^c]_p + [tA]_p U^c, added to zeroed E U^c and [tZ^c]_p.
template <class R>
__global__ __launch_bounds__(TPB) void k_np_gemv(const LayerDev *__restrict__ Ls) {
    const LayerDev &L = Ls[blockIdx.y];
    if (np_fused_row(L.N)) return;  // formed by k_np_row_pass
    const int np = L.np;
    const NpCvec o = np_cvec(L.M, L.K, np);
    R *cv = P<R>(L.cvec);
    const int64_t K = L.K;
    auto elem = [&](int64_t m, int64_t k, R (&v)[1 + MAXP]) {
        const int64_t e = m * K + k;
        const R E = ld(P<R>(L.E), e), uc = ld(cv + o.Uc, k);
        v[0] = mad(v[0], E, uc);
#pragma unroll
        for (int p = 0; p < MAXP; p++)
            if (p < np) v[1 + p] = mad(mad(v[1 + p], E, ld(cv + o.tb(p), k)), ld(P<R>(L.tA[p]), e), uc);
    };
    auto done = [&](int64_t m, R (&v)[1 + MAXP]) {
        atomic_add128(cv + o.EUc + m, v[0]);
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) atomic_add128(cv + o.tz(p) + m, v[1 + p]);
    };
    row_sweep<R, 1 + MAXP>(hw_grid(), L.M, K, elem, done);
}

hipError_t launch_np_gemv(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st) {
    LAUNCH_RING(eb, k_np_gemv, dim3(grid_items(max_items), n), dim3(TPB), st, L);
    return hipGetLastError();
}

// Eq. (5) per row i: [tZ^c]_p = [tC^c]_p + (E [tB^c]_p + [tA]_p U^c) + [Delta]_p (E U^c),
// [tD^c]_p = [tR^c]_p - [tZ^c]_p; F_CHECK: the compact check of D in
// accumulator form, acc_p = -sum chihat_i [tD^c]_p,i, acc_W = -sum chihat_i D^c_i.
template <class R>
__global__ __launch_bounds__(TPB) void k_np_compact_final(const LayerDev *__restrict__ Ls, int flags) {
    __shared__ R sh[ACC_W * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int np = L.np;
    const NpCvec o = np_cvec(L.M, L.K, np);
    R *cv = P<R>(L.cvec);
    R chk[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) chk[i] = Ring<R>::zero();
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < L.M; i += (int64_t)gridDim.x * TPB) {
        const R eu = ld(cv + o.EUc, i);
        const uint64_t x = Ring<R>::mod_s(sdraw(L.key[K_CHIHAT], (uint64_t)i));
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) {
            const R z = add(add(ld(cv + o.tc(p), i), ld(cv + o.tz(p), i)), mul64(eu, L.delta[p]));
            const R dd = sub(ld(cv + o.tr(p), i), z);
            st(cv + o.tz(p), i, z);
            st(cv + o.td(p), i, dd);
            if (flags & F_CHECK) chk[p] = mad64(chk[p], dd, x);
        }
        if (flags & F_CHECK) chk[MAXP] = mad64(chk[MAXP], ld(cv + o.Dc, i), x);
    }
    if (flags & F_CHECK) {
#pragma unroll
        for (int i = 0; i < ACC_W; i++) chk[i] = sub(Ring<R>::zero(), chk[i]);
        block_accumulate<ACC_W>(chk, sh, P<R>(L.acc) + 2 * ACC_W);
    }
}

hipError_t launch_np_compact_final(int eb, const LayerDev *L, int n, int flags, hipStream_t st) {
    LAUNCH_RING(eb, k_np_compact_final, dim3(4, n), dim3(TPB), st, L, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- checks
// Standalone Pi_BatchRec tag check (Fig. 1) of W = P - Q: y = layer * 3 + which,
// which = 0: E (X, A), 1: U (Y, B), 2: D (R, Z).
template <class R>
__global__ __launch_bounds__(TPB) void k_np_check_batch(const LayerDev *__restrict__ Ls, int which_mask) {
    __shared__ R sh[ACC_W * WAVES];
    const LayerDev &L = Ls[blockIdx.y / 3];
    const int which = blockIdx.y % 3, np = L.np;
    if (!((which_mask >> which) & 1)) return;
    int64_t n;
    u128 *const *tP;
    u128 *const *tQ;
    const R *W;
    uint64_t key;
    if (which == 0) {
        n = L.M * L.K; tP = L.tX; tQ = L.tA; W = P<R>(L.E); key = L.key[K_CHI_E];
    } else if (which == 1) {
        n = L.K * L.N; tP = L.tY; tQ = L.tB; W = P<R>(L.U); key = L.key[K_CHI_U];
    } else {
        n = L.M * L.N; tP = L.tR; tQ = L.tZ; W = P<R>(L.D); key = L.key[K_CHI_D];
    }
    if (blockIdx.x * (int64_t)TPB >= n) return;  // no elements for this workgroup
    R v[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) v[i] = Ring<R>::zero();
    for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const uint64_t c = Ring<R>::mod_s(sdraw(key, (uint64_t)e));
#pragma unroll
        for (int p = 0; p < MAXP; p++)
            if (p < np) v[p] = mad64(v[p], sub(ld(P<R>(tP[p]), e), ld(P<R>(tQ[p]), e)), c);
        v[MAXP] = mad64(v[MAXP], ld(W, e), c);
    }
    block_accumulate<ACC_W>(v, sh, P<R>(L.acc) + which * ACC_W);
}

hipError_t launch_np_check_batch(int eb, const LayerDev *L, int n, int which_mask, int64_t max_elems, hipStream_t st) {
    int g = grid_for(max_elems);
    if (g > 2048) g = 2048;
    LAUNCH_RING(eb, k_np_check_batch, dim3(g, 3 * n), dim3(TPB), st, L, which_mask);
    return hipGetLastError();
}

// Standalone compact check of D from the stored compact vectors.
template <class R>
__global__ __launch_bounds__(TPB) void k_np_check_compact(const LayerDev *__restrict__ Ls) {
    __shared__ R sh[ACC_W * WAVES];
    const LayerDev &L = Ls[blockIdx.y];
    const int np = L.np;
    const NpCvec o = np_cvec(L.M, L.K, np);
    const R *cv = P<R>(L.cvec);
    R v[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) v[i] = Ring<R>::zero();
    for (int64_t i = threadIdx.x; i < L.M; i += TPB) {
        const uint64_t c = Ring<R>::mod_s(sdraw(L.key[K_CHIHAT], (uint64_t)i));
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < np) v[p] = mad64(v[p], ld(cv + o.td(p), i), c);
        v[MAXP] = mad64(v[MAXP], ld(cv + o.Dc, i), c);
    }
    block_sum<ACC_W, WAVES>(v, sh);
    if (threadIdx.x == 0)
        for (int i = 0; i < ACC_W; i++) st(P<R>(L.acc), 2 * ACC_W + i, sub(Ring<R>::zero(), v[i]));
}

hipError_t launch_np_check_compact(int eb, const LayerDev *L, int n, hipStream_t st) {
    LAUNCH_RING(eb, k_np_check_compact, dim3(1, n), dim3(TPB), st, L);
    return hipGetLastError();
}

// cs[W][p] = acc[W ACC_W + p] - [Delta]_p acc[W ACC_W + MAXP]; accept iff
// sum_p cs[W][p] = 0 for every W.
template <class R>
__global__ __launch_bounds__(64) void k_np_finalize(const LayerDev *__restrict__ Ls, int n, ct_check_result *out) {
    const int l = blockIdx.x, lane = threadIdx.x;
    if (l >= n) return;
    const LayerDev &L = Ls[l];
    // the fused row pass's copies of the E sums, over the wavefront
    const unsigned long long *cells = rp_cells<R>(L);
    R e[ACC_W];
#pragma unroll
    for (int i = 0; i < ACC_W; i++) {
        e[i] = Ring<R>::zero();
        for (int s = lane; s < NP_RP_COPIES; s += 64) {
            R v;
            from_limbs(cells + 4 * ACC_W * s + 4 * i, v);
            e[i] = add(e[i], v);
        }
        e[i] = wave_sum(e[i]);
    }
    if (lane != 0) return;
    auto acc = [&](int w, int i) {
        const R v = ld(P<R>(L.acc), w * ACC_W + i);
        return w == 0 ? add(v, e[i]) : v;
    };
    ct_check_result r;
    for (int w = 0; w < 3; w++)
        for (int p = 0; p < CT_MAX_PARTIES; p++) r.cs[w][p] = ct_u128{0, 0};
    int ok = 1;
    for (int w = 0; w < 3; w++) {
        const R aw = acc(w, MAXP);
        R sum = Ring<R>::zero();
#pragma unroll
        for (int p = 0; p < MAXP; p++) if (p < L.np) {
            const R c = sub(acc(w, p), mul64(aw, L.delta[p]));
            r.cs[w][p] = Ring<R>::out(c);
            sum = add(sum, c);
        }
        if (Ring<R>::nonzero(sum)) ok = 0;
    }
    r.accept = ok;
    r.reserved = 0;
    out[L.out_index] = r;
}

hipError_t launch_np_finalize(int eb, const LayerDev *L, int n, ct_check_result *out, hipStream_t st) {
    LAUNCH_RING(eb, k_np_finalize, dim3(n), dim3(64), st, L, n, out);
    return hipGetLastError();
}

}  // namespace ct
