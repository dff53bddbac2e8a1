// ct_passes.h -- bodies of the bandwidth-bound stages of the two-party online
// phase (zeroing, constant terms of split products, the pass over M x K, the
// pass over M x N, the compact tag's final step and the check verdicts), each
// run as one workgroup of a grid (Grid): the stage kernels of ct_kernels.hip
// run them as themselves, the persistent launch of ct_gemm.hip as workgroups
// of its own grid.  The stage comments in ct_kernels.hip describe the passes.
#pragma once

#include "ct_sweep.h"

namespace ct {

// ---------------------------------------------------------------- zeroing
// what bit 0: the compressed vectors (cvec); bit 1: the check accumulators;
// bit 2: for layers with N <= SKINNY_MAX_N, [Z]_p = [C]_p (the row pass adds
// the products of each row segment atomically); bit 3: also [tZ]_p = [tC]_p.
template <class R>
__device__ __forceinline__ void zero_acc_body(const LayerDev *__restrict__ Ls, int what, const Grid &g) {
    const LayerDev &L = Ls[g.y];
    const int64_t t0 = (int64_t)g.x * TPB + threadIdx.x, stride = (int64_t)g.nx * TPB;
    if (what & 1) {
        const int64_t n = 3 * L.K + 10 * cvec_rows(L);
        for (int64_t e = t0; e < n; e += stride) st(P<R>(L.cvec), e, Ring<R>::zero());
    }
    if ((what & 2) && g.x == 0)  // ACC_PER_LAYER 16-byte elements whatever the ring
        for (int i = threadIdx.x; i < ACC_PER_LAYER; i += TPB) st(L.acc, i, u128{0, 0});
    if ((what & 4) && L.N <= SKINNY_MAX_N) {
        const int64_t n = L.M * L.N;
        for (int64_t e = t0; e < n; e += stride) {
            st(P<R>(L.Z[0]), e, ld(P<R>(L.C[0]), e));
            st(P<R>(L.Z[1]), e, ld(P<R>(L.C[1]), e));
            if (what & 8) {
                st(P<R>(L.tZ[0]), e, ld(P<R>(L.tC[0]), e));
                st(P<R>(L.tZ[1]), e, ld(P<R>(L.tC[1]), e));
            }
        }
    }
}

// Products whose K range is split add their partial results atomically onto
// the output, which first receives the product's constant term: [Z]_p = [C]_p
// (SPDZ2k also [tZ]_p = [tC]_p).  Only the split products are copied; the
// others add the constant term in the product's epilogue.
template <class R>
__device__ __forceinline__ void prob_base_body(const GemmProb *__restrict__ probs, const Grid &g) {
    const GemmProb &p = probs[g.y];
    if (!p.accumulate || !p.base) return;
    const int64_t n = (int64_t)p.M * p.N;
    for (int64_t e = (int64_t)g.x * TPB + threadIdx.x; e < n; e += (int64_t)g.nx * TPB)
        st(P<R>(p.out), e, ld(reinterpret_cast<const R *>(p.base), e));
}

// The pass over M x K of a layer that is not compressed along M: one
// wavefront per row segment of row_seg(M, K) elements (see ct_kernels.hip).
template <class R, int NS>
__device__ __forceinline__ void row_pass_body(const LayerDev &L, int flags, R (&chk)[3], const Grid &g) {
    const int lane = threadIdx.x & 63;
    const int64_t M = L.M, K = L.K, N = L.N;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT, spdz = flags & F_SPDZ;
    const bool skinny = NS > 0;
    const CvecOff o = cvec_off(M, K);
    const R *Uc = P<R>(L.cvec) + o.Uc, *tBc0 = P<R>(L.cvec) + o.tBc0, *tBc1 = P<R>(L.cvec) + o.tBc1;
    const uint64_t kce = L.key[K_CHI_E];
    const uint64_t d0 = L.delta[0], d1 = L.delta[1];
    R *AE0 = P<R>(L.work), *tAE0 = P<R>(L.work) + M * K, *tAE1 = P<R>(L.work) + 2 * M * K;
    const int64_t seg = row_seg(M, K), items = M * ((K + seg - 1) / seg);
    const int64_t wave_id = ((int64_t)g.x * TPB + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)g.nx * TPB) >> 6;
    // segment-major order: the wavefronts in flight share one segment of k,
    // so the K-long vectors they read (U^c, [tB^c]_p; U, [B]_p of skinny
    // layers) stay in L2 while the M x K arrays stream through
    for (int64_t it = wave_id; it < items; it += nwaves) {
        const int64_t sg = it / M, m = it - sg * M, k0 = sg * seg;
        const int64_t k1 = k0 + seg < K ? k0 + seg : K;
        // compact: E U^c, E tB^c_0, E tB^c_1, tA_0 U^c, tA_1 U^c
        R cp[5] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
        // skinny: Z_0, Z_1 (and SPDZ2k tZ_0, tZ_1) row products per column
        R z0[NS > 0 ? NS : 1], z1[NS > 0 ? NS : 1], t0[NS > 0 ? NS : 1], t1[NS > 0 ? NS : 1];
#pragma unroll
        for (int j = 0; j < (NS > 0 ? NS : 1); j++) z0[j] = z1[j] = t0[j] = t1[j] = Ring<R>::zero();
        const int64_t rb = m * K;
        // the elements of one M x K position: shares of X, A and their tags
        struct In {
            R a0, a1, x0, x1, ta0, ta1, tx0, tx1;
        };
        const bool need_ta = check || compact || spdz;
        auto load = [&](int64_t e, In &v) {
            // the arrays are streamed, except [A]_1 of a matrix-core layer,
            // which k_pack reads next
            v.a0 = ld_nt(P<R>(L.A[0]), e);
            v.a1 = skinny ? ld_nt(P<R>(L.A[1]), e) : ld(P<R>(L.A[1]), e);
            v.x0 = ld_nt(P<R>(L.X[0]), e);
            v.x1 = ld_nt(P<R>(L.X[1]), e);
            v.ta0 = v.ta1 = v.tx0 = v.tx1 = Ring<R>::zero();
            if (need_ta) {
                v.ta0 = ld_nt(P<R>(L.tA[0]), e);
                v.ta1 = ld_nt(P<R>(L.tA[1]), e);
            }
            if (check) {
                v.tx0 = ld_nt(P<R>(L.tX[0]), e);
                v.tx1 = ld_nt(P<R>(L.tX[1]), e);
            }
        };
        auto use = [&](int64_t k, const In &v) {
            const int64_t e = rb + k;
            const R E = add(sub(v.x0, v.a0), sub(v.x1, v.a1));
            // E of a layer whose products are formed here is not read again
            // in the step; a matrix-core layer's is packed next
            if (skinny) st_nt(P<R>(L.E), e, E);
            else st(P<R>(L.E), e, E);
            if (check) {
                const uint64_t x = Ring<R>::mod_s(sdraw(kce, (uint64_t)e));
                chk[0] = mad64(chk[0], sub(v.tx0, v.ta0), x);
                chk[1] = mad64(chk[1], sub(v.tx1, v.ta1), x);
                chk[2] = mad64(chk[2], E, x);
            }
            if (compact) {
                const R uc = ld(Uc, k);
                cp[0] = mad(cp[0], E, uc);
                cp[1] = mad(cp[1], E, ld(tBc0, k));
                cp[2] = mad(cp[2], E, ld(tBc1, k));
                cp[3] = mad(cp[3], v.ta0, uc);
                cp[4] = mad(cp[4], v.ta1, uc);
            }
            if constexpr (!skinny) {
                // folded left operands of the matrix-core products:
                //   [Z]_0 = [C]_0 + E [B]_0 + (A_0 + E) U,
                //   [tZ]_p = [tC]_p + E [tB]_p + ([tA]_p + [Delta]_p E) U
                st(AE0, e, add(v.a0, E));
                if (spdz) {
                    st(tAE0, e, add(v.ta0, mul64(E, d0)));
                    st(tAE1, e, add(v.ta1, mul64(E, d1)));
                }
            } else {
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    if (j < N) {
                        const int64_t kn = k * N + j;
                        const R u = ld(P<R>(L.U), kn);
                        z0[j] = mad(mad(z0[j], E, add(ld(P<R>(L.B[0]), kn), u)), v.a0, u);
                        z1[j] = mad(mad(z1[j], E, ld(P<R>(L.B[1]), kn)), v.a1, u);
                        if (spdz) {
                            t0[j] = mad(mad(t0[j], E, add(ld(P<R>(L.tB[0]), kn), mul64(u, d0))), v.ta0, u);
                            t1[j] = mad(mad(t1[j], E, add(ld(P<R>(L.tB[1]), kn), mul64(u, d1))), v.ta1, u);
                        }
                    }
                }
            }
        };
        // every load of the element is issued before the store of E (which
        // the compiler may not move loads across).  Two elements per lane at
        // a time would double the loads in flight but costs registers: the
        // skinny pass then runs 3 wavefronts per SIMD instead of 4, and is
        // slower.
        for (int64_t k = k0 + lane; k < k1; k += 64) {
            In v;
            load(rb + k, v);
            use(k, v);
        }
        if (compact) {
            // the partial compact tags E tB^c_p + tA_p U^c summed per lane
            // first: three wavefront reductions for the five row products
            const R val[3] = {wave_sum(cp[0]), wave_sum(add(cp[1], cp[3])), wave_sum(add(cp[2], cp[4]))};
            if (lane == 0) {
                // E U^c, and the partial compact tags (k_compact_final adds
                // [tC^c]_p and [Delta]_p E U^c); the three atomics in flight together
                R *const cell[3] = {P<R>(L.cvec) + o.EUc + m, P<R>(L.cvec) + o.tZc0 + m, P<R>(L.cvec) + o.tZc1 + m};
                const bool ok[3] = {true, true, true};
                atomic_add128_n<3>(cell, val, ok);
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
                        R *const cell[4] = {P<R>(L.Z[0]) + mn, P<R>(L.Z[1]) + mn, P<R>(L.tZ[0]) + mn,
                                            P<R>(L.tZ[1]) + mn};
                        const R val[4] = {z0[j], z1[j], t0[j], t1[j]};
                        const bool ok[4] = {true, true, spdz, spdz};
                        atomic_add128_n<4>(cell, val, ok);
                    }
                }
            }
        }
    }
}

// One layer's row pass (variant NS, not compressed along M) as workgroup g,
// and the workgroup's check sums of E into its copy of the accumulators.
template <class R, int NS>
__device__ __forceinline__ void row_pass_layer(const LayerDev *__restrict__ Ls, int flags, const Grid &g) {
    const LayerDev &L = Ls[g.y];
    if (row_variant(L.N) != NS || ((flags & F_COMPACT) && L.cm)) return;
    R chk[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    row_pass_body<R, NS>(L, flags, chk, g);
    if (flags & F_CHECK)
        wave_accumulate_limbs<3>(chk, rp_cells<R>(L) + 12 * ((((unsigned)g.x * TPB + threadIdx.x) >> 6) % RP_COPIES));
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
template <class R>
__device__ __forceinline__ void truncate_out(const LayerDev &L, int64_t e, R D) {
    const uint64_t df = Ring<R>::mod_k(D) >> L.f;
    st(P<R>(L.Zf[0]), e, sub(ld(P<R>(L.Rf[0]), e), Ring<R>::small(df)));
    st(P<R>(L.Zf[1]), e, ld(P<R>(L.Rf[1]), e));
    st(P<R>(L.tZf[0]), e, sub(ld(P<R>(L.tRf[0]), e), mul64(Ring<R>::small(L.delta[0]), df)));
    st(P<R>(L.tZf[1]), e, sub(ld(P<R>(L.tRf[1]), e), mul64(Ring<R>::small(L.delta[1]), df)));
}

template <class R>
__device__ __forceinline__ void post_body(const LayerDev *__restrict__ Ls, int flags, const Grid &g) {
    __shared__ R sh[3 * WAVES];
    const LayerDev &L = Ls[g.y];
    const int64_t M = L.M, N = L.N;
    const bool check = flags & F_CHECK, compact = flags & F_COMPACT;
    const uint64_t kchi = L.key[K_CHI], kcd = L.key[K_CHI_D];
    R chk[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    if (compact) {
        const bool cm = L.cm;
        const CvecOff o = cvec_off(cvec_rows(L), L.K);
        auto elem = [&](int64_t r, int64_t c, R (&v)[5]) {
            const int64_t e = r * N + c;
            const R D = add(sub(ld(P<R>(L.R[0]), e), ld(P<R>(L.Z[0]), e)), sub(ld(P<R>(L.R[1]), e), ld(P<R>(L.Z[1]), e)));
            st(P<R>(L.D), e, D);
            if (L.f > 0) truncate_out(L, e, D);
            const R tr0 = ld(P<R>(L.tR[0]), e), tr1 = ld(P<R>(L.tR[1]), e);
            st(P<R>(L.tZ[0]), e, sub(tr0, mul64(D, L.delta[0])));
            st(P<R>(L.tZ[1]), e, sub(tr1, mul64(D, L.delta[1])));
            // combiner of the compressed index: the column (along N) or the row (along M)
            const uint64_t x = Ring<R>::mod_s(sdraw(kchi, (uint64_t)(cm ? r : c)));
            v[0] = mad64(v[0], D, x);
            v[1] = mad64(v[1], tr0, x);
            v[2] = mad64(v[2], tr1, x);
            v[3] = mad64(v[3], ld(P<R>(L.tC[0]), e), x);
            v[4] = mad64(v[4], ld(P<R>(L.tC[1]), e), x);
        };
        // each sweep hands its partial sums for entry i (a row, or a column)
        auto done = [&](int64_t i, R (&v)[5]) {
            add_cells<5>(P<R>(L.cvec), {o.Dc, o.tRc0, o.tRc1, o.tCc0, o.tCc1}, i, v);
        };
        if (cm) col_sweep<R, 5>(g, M, N, elem, done);
        else row_sweep<R, 5>(g, M, N, elem, done);
    } else {
        const int64_t n = M * N;
        for (int64_t e = (int64_t)g.x * TPB + threadIdx.x; e < n; e += (int64_t)g.nx * TPB) {
            const R z0 = ld(P<R>(L.Z[0]), e), z1 = ld(P<R>(L.Z[1]), e);
            const R D = add(sub(ld(P<R>(L.R[0]), e), z0), sub(ld(P<R>(L.R[1]), e), z1));
            st(P<R>(L.D), e, D);
            if (L.f > 0) truncate_out(L, e, D);
            if (check) {
                const uint64_t x = Ring<R>::mod_s(sdraw(kcd, (uint64_t)e));
                chk[0] = mad64(chk[0], sub(ld(P<R>(L.tR[0]), e), ld(P<R>(L.tZ[0]), e)), x);
                chk[1] = mad64(chk[1], sub(ld(P<R>(L.tR[1]), e), ld(P<R>(L.tZ[1]), e)), x);
                chk[2] = mad64(chk[2], D, x);
            }
        }
        if (check) block_accumulate<3>(chk, sh, P<R>(L.acc) + 6);
    }
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
__device__ __forceinline__ void compact_final_body(const LayerDev *__restrict__ Ls, int flags, const Grid &g) {
    __shared__ R sh[3 * WAVES];
    const LayerDev &L = Ls[g.y];
    const int64_t M = cvec_rows(L);
    const CvecOff o = cvec_off(M, L.K);
    R *c = P<R>(L.cvec);
    R v[3] = {Ring<R>::zero(), Ring<R>::zero(), Ring<R>::zero()};
    for (int64_t i = (int64_t)g.x * TPB + threadIdx.x; i < M; i += (int64_t)g.nx * TPB) {
        const R eu = ld(c + o.EUc, i);
        const R z0 = add(add(ld(c + o.tCc0, i), ld(c + o.tZc0, i)), mul64(eu, L.delta[0]));
        const R z1 = add(add(ld(c + o.tCc1, i), ld(c + o.tZc1, i)), mul64(eu, L.delta[1]));
        const R dd0 = sub(ld(c + o.tRc0, i), z0), dd1 = sub(ld(c + o.tRc1, i), z1);
        st(c + o.tZc0, i, z0);
        st(c + o.tZc1, i, z1);
        st(c + o.tDc0, i, dd0);
        st(c + o.tDc1, i, dd1);
        if (flags & F_CHECK) {
            const uint64_t x = Ring<R>::mod_s(sdraw(L.key[K_CHIHAT], (uint64_t)i));
            v[0] = mad64(v[0], dd0, x);
            v[1] = mad64(v[1], dd1, x);
            v[2] = mad64(v[2], ld(c + o.Dc, i), x);
        }
    }
    if (flags & F_CHECK) {
#pragma unroll
        for (int i = 0; i < 3; i++) v[i] = sub(Ring<R>::zero(), v[i]);
        block_accumulate<3>(v, sh, P<R>(L.acc) + 6);
    }
}

// cs[W][p] = acc[3W + p] - [Delta]_p acc[3W + 2]; accept iff every cs sum is 0.
template <class R>
__device__ __forceinline__ void finalize_body(const LayerDev *__restrict__ Ls, int n, ct_check_result *out, int l) {
    const int lane = threadIdx.x & 63;
    if (l >= n) return;
    const LayerDev &L = Ls[l];
    // the row pass's copies of the E sums, over the wavefront (zero where
    // another kernel accumulated them)
    const unsigned long long *cells = rp_cells<R>(L);
    R e[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        e[i] = Ring<R>::zero();
        for (int s = lane; s < RP_COPIES; s += 64) {
            R v;
            from_limbs(cells + 12 * s + 4 * i, v);
            e[i] = add(e[i], v);
        }
        e[i] = wave_sum(e[i]);
    }
    if (lane != 0) return;
    for (int i = 0; i < 3; i++) e[i] = add(e[i], ld(P<R>(L.acc), i));
    int ok = 1;
    ct_check_result r;
    for (int w = 0; w < 3; w++)
        for (int p = 0; p < CT_MAX_PARTIES; p++) r.cs[w][p] = ct_u128{0, 0};
    for (int w = 0; w < 3; w++) {
        const R aw = w == 0 ? e[2] : ld(P<R>(L.acc), 3 * w + 2);
        R c[2];
        for (int p = 0; p < 2; p++) {
            c[p] = sub(w == 0 ? e[p] : ld(P<R>(L.acc), 3 * w + p), mul64(aw, L.delta[p]));
            r.cs[w][p] = Ring<R>::out(c[p]);
        }
        if (Ring<R>::nonzero(add(c[0], c[1]))) ok = 0;
    }
    r.accept = ok;
    r.reserved = 0;
    out[L.out_index] = r;
}

}  // namespace ct
