/*
 * ct_oracle.c -- plain, slow CPU oracle for the linear-layer hot path of
 * CompactTag (arXiv 2311.04406): two to five parties of SPDZ2k-style MPC over
 * the value ring Z_{2^k} with shares and tags in Z_{2^{k+s}} and key shares in
 * Z_{2^s}, for the two parameter sets of Sec. 4.1: k = s = 64 (Z_{2^128}) and
 * k = s = 32 (Z_{2^64}).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this file.  It shares no code with the
 * GPU library and must never be used as a fallback for it.
 *
 * Everything is naive loops over `unsigned __int128`, whose arithmetic wraps
 * modulo 2^128; with k + s = 64 every stored value is reduced mod 2^64 (a ring
 * homomorphism, so reducing at each store equals computing in Z_{2^64}), and
 * the operations that are not ring operations -- the key, combiner and input
 * draws, the truncation -- reduce explicitly.  Each step follows the
 * paper in order:
 *   - authenticated sharing, Sec. 2.4 and Eq. (1);
 *   - the preprocessing functionalities F_Rand and F_MAC, Appendix A;
 *   - Pi_BatchRec (Fig. 1): open and tag check;
 *   - Pi_MatMul (Fig. 2, Eqs. (2)-(3)): the SPDZ2k baseline;
 *   - Pi_Compress (Fig. 4), Pi_OptMAC (Fig. 5), the compact tag of
 *     Eq. (5) and Pi_CompactMatMul (Fig. 7), along N or along M;
 *   - truncation for f > 0: OptMAC&Trunc (Fig. 6) / Pi_Truncation (Fig. 3);
 *   - convolutions as im2col products (Eq. (4)) opened on the input's shape;
 *   - n parties (the appendix on scaling with parties).
 * Readings where the paper is ambiguous (integer key sum, the party that adds
 * public value terms, D opened mod 2^{k+s}, E*U inside the compact tag, check
 * modulus 2^{k+s}) are the ones listed in the design notes and in the file
 * comments below.
 */
#include "ct_oracle.h"

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Ring multiplications performed so far by this thread; the tag accounting of
 * Sec. 3.4.3 is read off this counter around the tag computations.  Both this
 * counter and the ring width below are per thread, so row ranges of a layer
 * (or different layers) can run on several threads at once. */
static _Thread_local uint64_t g_mults;

/* k = s of the current call on this thread: 64 (ring Z_{2^128}) or 32 (ring Z_{2^64}). */
static _Thread_local int64_t g_kbits = 64;

void or_set_kbits(int64_t kbits) { g_kbits = kbits == 32 ? 32 : 64; }

/* x mod 2^s for a draw used as a key share or a combiner (s = k) */
static uint64_t mod_s(uint64_t x) { return g_kbits == 32 ? (x & 0xFFFFFFFFULL) : x; }
/* v mod 2^k: the value of a lifted element */
static uint64_t mod_k(u128 v) { return g_kbits == 32 ? (uint64_t)(uint32_t)v : (uint64_t)v; }

/* ------------------------------------------------------------------ */
/* (lo, hi) limb storage; stores reduce mod 2^{k+s}                      */

static inline u128 ld(const uint64_t *p, int64_t i) {
    return (u128)p[2 * i] | ((u128)p[2 * i + 1] << 64);
}
static inline void st(uint64_t *p, int64_t i, u128 v) {
    p[2 * i] = (uint64_t)v;
    p[2 * i + 1] = g_kbits == 32 ? 0 : (uint64_t)(v >> 64);
}
static uint64_t *alloc128(int64_t n) {
    uint64_t *p = (uint64_t *)calloc((size_t)(n > 0 ? n : 1) * 2, sizeof(uint64_t));
    if (!p) abort();
    return p;
}

/* ------------------------------------------------------------------ */
/* F_Rand / F_MAC stand-in: counter-based SplitMix64                    */
/* (Steele, Lea and Flood, "Fast splittable pseudorandom number         */
/*  generators", OOPSLA 2014).  The i-th draw (0-based) of a stream is   */
/*  the (i+1)-th output of SplitMix64 started at the stream key.         */

#define OR_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t or_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_stream_key(uint64_t seed, uint64_t stream) { return or_mix64(seed ^ or_mix64(stream)); }

uint64_t or_draw(uint64_t seed, uint64_t stream, uint64_t i) {
    return or_mix64(or_stream_key(seed, stream) + (i + 1) * OR_GAMMA);
}

void or_draw_many(uint64_t seed, uint64_t stream, uint64_t first, int64_t n, uint64_t *out) {
    for (int64_t i = 0; i < n; i++) out[i] = or_draw(seed, stream, first + (uint64_t)i);
}

static uint64_t stream_of(uint64_t layer_id, uint64_t purpose) { return (layer_id << 16) | purpose; }

/* element e of a 128-bit stream is draw(2e) + 2^64 * draw(2e+1) */
static u128 draw128(uint64_t seed, uint64_t stream, uint64_t e) {
    return (u128)or_draw(seed, stream, 2 * e) | ((u128)or_draw(seed, stream, 2 * e + 1) << 64);
}

/* F_MAC Initialize: key shares [Delta]_p uniform in Z_{2^s} (the draw mod 2^s). */
void or_key_shares_n(uint64_t key_seed, int64_t kbits, int64_t parties, uint64_t *delta) {
    for (int64_t p = 0; p < parties; p++) {
        const uint64_t x = or_draw(key_seed, stream_of(OR_GLOBAL_LAYER, OR_P_KEY + (uint64_t)p), 0);
        delta[p] = kbits == 32 ? (x & 0xFFFFFFFFULL) : x;
    }
}
void or_key_shares_k(uint64_t key_seed, int64_t kbits, uint64_t delta[2]) { or_key_shares_n(key_seed, kbits, 2, delta); }
void or_key_shares(uint64_t key_seed, uint64_t delta[2]) { or_key_shares_k(key_seed, 64, delta); }

/* parties of a descriptor */
static int parties_of(const or_desc *d) {
    if (d->parties == 0) return 2;
    if (d->parties < 2 || d->parties > OR_MAX_PARTIES) abort();
    return (int)d->parties;
}

/* combiner draws: uniform in Z_{2^s} */
static void draw_chi(uint64_t seed, uint64_t stream, uint64_t first, int64_t n, uint64_t *out) {
    or_draw_many(seed, stream, first, n, out);
    for (int64_t i = 0; i < n; i++) out[i] = mod_s(out[i]);
}

/* The key used in every tag relation is the integer sum of the key shares
 * (< n 2^s), taken mod 2^{k+s}; see the reading of Sec. 2.4 in the design notes. */
static u128 key_sum(const uint64_t *delta, int np) {
    u128 s = 0;
    for (int p = 0; p < np; p++) s += (u128)delta[p];
    return s;
}

/* ------------------------------------------------------------------ */
/* building blocks                                                      */

/* out = P * Q mod 2^128 for P (M x K), Q (K x N); a plain triple loop. */
void or_matmul(int64_t M, int64_t K, int64_t N, const uint64_t *P, const uint64_t *Q, uint64_t *out) {
    u128 *acc = (u128 *)calloc((size_t)(N > 0 ? N : 1), sizeof(u128));
    if (!acc) abort();
    for (int64_t i = 0; i < M; i++) {
        memset(acc, 0, (size_t)N * sizeof(u128));
        for (int64_t k = 0; k < K; k++) {
            u128 a = ld(P, i * K + k);
            for (int64_t j = 0; j < N; j++) acc[j] += a * ld(Q, k * N + j);
            g_mults += (uint64_t)N;
        }
        for (int64_t j = 0; j < N; j++) st(out, i * N + j, acc[j]);
    }
    free(acc);
}

/* Pi_Compress (Fig. 4, step 1): M^c = M * chi, chi in Z_{2^s}^{N x 1}. */
void or_compress(int64_t rows, int64_t N, const uint64_t *Mx, const uint64_t *chi, uint64_t *out) {
    for (int64_t i = 0; i < rows; i++) {
        u128 s = 0;
        for (int64_t j = 0; j < N; j++) s += ld(Mx, i * N + j) * (u128)chi[j];
        g_mults += (uint64_t)N;
        st(out, i, s);
    }
}

/* Pi_Compress along the other dimension (Sec. 2.2 leaves the compressed
 * dimension open): M^c = chi^T * M for M (rows x N), chi in Z_{2^s}^{rows x 1};
 * entry j combines column j of M. */
void or_compress_rows(int64_t rows, int64_t N, const uint64_t *Mx, const uint64_t *chi, uint64_t *out) {
    for (int64_t j = 0; j < N; j++) {
        u128 s = 0;
        for (int64_t i = 0; i < rows; i++) s += (u128)chi[i] * ld(Mx, i * N + j);
        g_mults += (uint64_t)rows;
        st(out, j, s);
    }
}

/* Pi_BatchRec tag check (Fig. 1, tag-check steps 2-3), one party's share:
 *   [CS] = [tag W] (.) chi - [Delta]_p * (W (.) chi),  cs_p = sum of all entries of [CS],
 * everything mod 2^{k+s}. */
void or_batchrec_cs(int64_t n, const uint64_t *W, const uint64_t *tW, const uint64_t *chi,
                    uint64_t delta_p, uint64_t out[2]) {
    u128 cs = 0;
    for (int64_t e = 0; e < n; e++) {
        u128 CS = ld(tW, e) * (u128)chi[e] - (u128)delta_p * (ld(W, e) * (u128)chi[e]);
        cs += CS;
    }
    st(out, 0, cs);
}

/* Pi_CompactMatMul verification, steps 3-5 (Fig. 7), one party's share:
 *   [CS] = [Delta]_p * D^c;  [CS] = [CS] (.) chihat - [tag D^c] (.) chihat;  cs_p = sum_i [CS]_i.
 * Reduced mod 2^{k+s} (reading of the k+2s modulus in the design notes). */
void or_compact_cs(int64_t rows, const uint64_t *Dc, const uint64_t *tDc, const uint64_t *chihat,
                   uint64_t delta_p, uint64_t out[2]) {
    u128 cs = 0;
    for (int64_t i = 0; i < rows; i++) {
        u128 CS = (u128)delta_p * ld(Dc, i);
        CS = CS * (u128)chihat[i] - ld(tDc, i) * (u128)chihat[i];
        cs += CS;
    }
    st(out, 0, cs);
}

/* ------------------------------------------------------------------ */
/* preprocessing: a trusted dealer in place of F_MAC Auth               */

/* Authenticated n-party sharing of one lifted value (Sec. 2.4): the value and
 * tag shares of parties 0..n-2 are fresh draws (party p from the streams of
 * purpose VSH / TSH + object + 256 p), the last party's complete the sums
 *   sum_p [v]_p = v~,   sum_p [t]_p = Delta~ * v~   (mod 2^{k+s}). */
static void auth_share(int np, u128 lift, u128 dsum, uint64_t seed, uint64_t layer_id, int obj, uint64_t e,
                       uint64_t *const v[], uint64_t *const t[], int64_t at) {
    u128 sv = 0, stg = 0;
    for (int p = 0; p < np - 1; p++) {
        const uint64_t shift = (uint64_t)p << 8;
        const u128 a = draw128(seed, stream_of(layer_id, OR_P_VSH + (uint64_t)obj + shift), e);
        const u128 b = draw128(seed, stream_of(layer_id, OR_P_TSH + (uint64_t)obj + shift), e);
        st(v[p], at, a);
        st(t[p], at, b);
        sv += a;
        stg += b;
    }
    st(v[np - 1], at, lift - sv);
    st(t[np - 1], at, dsum * lift - stg);
}

enum { OBJ_X = 1, OBJ_Y = 2, OBJ_A = 3, OBJ_B = 4, OBJ_C = 5, OBJ_R = 6, OBJ_RF = 7 };

/* ------------------------------------------------------------------ */
/* convolution as a matrix product (Eq. (4))                             */

static int64_t conv_out(int64_t in, const or_desc *d) {
    return (in + 2 * d->conv_pad - d->conv_k) / d->conv_stride + 1;
}

/* A convolution layer's K and N must be those of its geometry. */
static void conv_validate(const or_desc *d) {
    if (d->conv_c <= 0) return;
    if (d->conv_k < 1 || d->conv_stride < 1 || d->conv_pad < 0 || d->conv_h + 2 * d->conv_pad < d->conv_k ||
        d->conv_w + 2 * d->conv_pad < d->conv_k || d->K != d->conv_c * d->conv_k * d->conv_k ||
        d->N != conv_out(d->conv_h, d) * conv_out(d->conv_w, d))
        abort();
}

int64_t or_right_len(const or_desc *d) {
    return d->conv_c > 0 ? d->conv_c * d->conv_h * d->conv_w : d->K * d->N;
}

/* Row k = (c kh + dy) kw + dx of the im2col matrix lists, for every output
 * position n = y Wo + x, the input element under kernel tap (dy, dx):
 * (c, y s + dy - p, x s + dx - p), zero where that falls in the padding. */
void or_im2col(const or_desc *d, const uint64_t *in, uint64_t *out) {
    conv_validate(d);
    const int64_t kk = d->conv_k, Ho = conv_out(d->conv_h, d), Wo = conv_out(d->conv_w, d);
    for (int64_t c = 0; c < d->conv_c; c++)
        for (int64_t dy = 0; dy < kk; dy++)
            for (int64_t dx = 0; dx < kk; dx++) {
                const int64_t k = (c * kk + dy) * kk + dx;
                for (int64_t y = 0; y < Ho; y++)
                    for (int64_t x = 0; x < Wo; x++) {
                        const int64_t iy = y * d->conv_stride + dy - d->conv_pad;
                        const int64_t ix = x * d->conv_stride + dx - d->conv_pad;
                        u128 v = 0;
                        if (iy >= 0 && iy < d->conv_h && ix >= 0 && ix < d->conv_w)
                            v = ld(in, (c * d->conv_h + iy) * d->conv_w + ix);
                        st(out, k * d->N + y * Wo + x, v);
                    }
            }
}

/* An input value of Z_{2^k}: the draw mod 2^k, or with in_bits in 1..k-1 a
 * signed in_bits-bit integer (the top in_bits of those k bits, sign-extended)
 * in two's complement -- a stand-in for fixed-point encodings.  Lifted with
 * zero upper bits. */
static u128 input_lift(uint64_t draw, int64_t in_bits) {
    if (g_kbits == 32) {
        const uint32_t x = (uint32_t)draw;
        if (in_bits <= 0 || in_bits >= 32) return (u128)x;
        return (u128)(uint32_t)((int32_t)x >> (32 - in_bits));
    }
    if (in_bits <= 0 || in_bits >= 64) return (u128)draw;
    return (u128)(uint64_t)((int64_t)draw >> (64 - in_bits));
}

/* Preprocessing of Fig. 7 (Beaver matrix triple A, B, C = A*B and the mask R),
 * plus, when with_inputs is set, authenticated shares of the inputs X and Y.
 * Inputs are values of Z_{2^k} lifted with zero upper bits; A, B, R are
 * uniform in Z_{2^{k+s}}; C~ = A~ * B~ mod 2^{k+s}.  With f > 0 also the
 * truncated mask of Figs. 3 and 6, R^f = (R mod 2^k) / 2^f (an integer below
 * 2^{k-f}), lifted with a uniform upper limb and authenticated like the rest. */
void or_deal(const or_desc *d, const uint64_t *delta, int with_inputs, or_bufs *b) {
    or_set_kbits(d->kbits);
    const int64_t M = d->M, K = d->K, N = d->N, r0 = d->r0, rows = d->r1 - d->r0;
    const uint64_t seed = d->seed, lid = d->layer_id;
    const int np = parties_of(d);
    const u128 dsum = key_sum(delta, np);
    (void)M;
    conv_validate(d);
    /* the right operand's buffers: K x N, or for a convolution the input's
     * shape, whose im2col matrix (Eq. (4)) is the product's right operand */
    const int64_t nr = or_right_len(d);

    uint64_t *At = alloc128(rows * K), *Bt = alloc128(nr), *Ct = alloc128(rows * N);
    for (int64_t i = 0; i < rows; i++)
        for (int64_t k = 0; k < K; k++)
            st(At, i * K + k, draw128(seed, stream_of(lid, OR_P_LIFT_A), (uint64_t)((r0 + i) * K + k)));
    for (int64_t e = 0; e < nr; e++) st(Bt, e, draw128(seed, stream_of(lid, OR_P_LIFT_B), (uint64_t)e));
    if (d->conv_c > 0) {
        uint64_t *Bx = alloc128(K * N);
        or_im2col(d, Bt, Bx);
        or_matmul(rows, K, N, At, Bx, Ct);
        free(Bx);
    } else {
        or_matmul(rows, K, N, At, Bt, Ct);
    }

    for (int64_t i = 0; i < rows; i++)
        for (int64_t k = 0; k < K; k++) {
            int64_t at = i * K + k;
            uint64_t e = (uint64_t)((r0 + i) * K + k);
            if (with_inputs) {
                u128 x = input_lift(or_draw(seed, stream_of(lid, OR_P_LIFT_X), e), d->in_bits);
                auth_share(np, x, dsum, seed, lid, OBJ_X, e, b->X, b->tX, at);
            }
            auth_share(np, ld(At, at), dsum, seed, lid, OBJ_A, e, b->A, b->tA, at);
        }
    for (int64_t e = 0; e < nr; e++) {
        if (with_inputs) {
            u128 y = input_lift(or_draw(seed, stream_of(lid, OR_P_LIFT_Y), (uint64_t)e), d->in_bits);
            auth_share(np, y, dsum, seed, lid, OBJ_Y, (uint64_t)e, b->Y, b->tY, e);
        }
        auth_share(np, ld(Bt, e), dsum, seed, lid, OBJ_B, (uint64_t)e, b->B, b->tB, e);
    }
    for (int64_t i = 0; i < rows; i++)
        for (int64_t j = 0; j < N; j++) {
            int64_t at = i * N + j;
            uint64_t e = (uint64_t)((r0 + i) * N + j);
            u128 r = draw128(seed, stream_of(lid, OR_P_LIFT_R), e);
            auth_share(np, ld(Ct, at), dsum, seed, lid, OBJ_C, e, b->C, b->tC, at);
            auth_share(np, r, dsum, seed, lid, OBJ_R, e, b->R, b->tR, at);
            if (d->f > 0) {
                const uint64_t up = mod_s(or_draw(seed, stream_of(lid, OR_P_LIFT_RF), e));
                u128 rf = (u128)(mod_k(r) >> d->f) | ((u128)up << g_kbits);
                auth_share(np, rf, dsum, seed, lid, OBJ_RF, e, b->Rf, b->tRf, at);
            }
        }
    free(At);
    free(Bt);
    free(Ct);
}

/* ------------------------------------------------------------------ */
/* online phase (what the GPU library calls tag_linear)                 */

/* Pi_BatchRec open (Fig. 1, steps 1-3) of W = P - Q for authenticated P, Q:
 * each party's share [W]_p = [P]_p - [Q]_p is broadcast and W = sum_p [W]_p
 * mod 2^{k+s}.  The zero mask of Fig. 1 is omitted: Q is a uniform Beaver mask. */
/* Pi_BatchRec open of W = P - Q: party p broadcasts [P]_p - [Q]_p, and W is
 * the sum of the broadcasts. */
static void open_diff(int np, int64_t n, uint64_t *const P[], uint64_t *const Q[], uint64_t *W) {
    for (int64_t e = 0; e < n; e++) {
        u128 w = 0;
        for (int p = 0; p < np; p++) w += ld(P[p], e) - ld(Q[p], e);
        st(W, e, w);
    }
}

static void add_into(int64_t n, uint64_t *acc, const uint64_t *x) {
    for (int64_t e = 0; e < n; e++) st(acc, e, ld(acc, e) + ld(x, e));
}

/* The compact tag with the compression taken along M instead of N (the
 * compressed dimension is a free choice, Sec. 2.2; the cost count of
 * Sec. 3.4.3 with the roles of M and N exchanged is 4MN + 2MK + 3KN + N
 * multiplications, fewer than 4MN + 2KN + 3MK + M exactly when M > N).
 * Fig. 7 steps 5-7 with every compression W^c = chi^T W, chi in Z_{2^s}^{M x 1}:
 * Eq. (5) multiplied by chi^T from the left is
 *   [tZ^c]_p = [tC^c]_p + E^c [tB]_p + [tA^c]_p U + [Delta]_p (E^c U),
 *   [tD^c]_p = [tR^c]_p - [tZ^c]_p,
 * with E^c = chi^T E and [tA^c]_p = chi^T [tA]_p of length K and every other
 * compressed vector of length N.  The public vectors E^c, D~^c and E^c U are
 * charged to each party. */
static void compact_rows(const or_desc *d, const uint64_t *delta, or_bufs *b, const uint64_t *opt) {
    const int64_t M = d->M, K = d->K, N = d->N;
    const int np = parties_of(d);
    if (d->r0 != 0 || d->r1 != M) abort();
    uint64_t *chi = (uint64_t *)malloc((size_t)(M > 0 ? M : 1) * 8);
    uint64_t *v = alloc128(N);
    if (!chi) abort();
    draw_chi(d->seed, stream_of(d->layer_id, OR_P_CHI), 0, M, chi);
    uint64_t m_pub = g_mults;
    or_compress_rows(M, K, b->E, chi, b->Ec);
    or_compress_rows(M, N, b->D, chi, b->Dc);
    or_matmul(1, K, N, b->Ec, b->U, b->EUc);
    const uint64_t pub_mults = g_mults - m_pub;
    for (int p = 0; p < np; p++) {
        uint64_t m0 = g_mults;
        or_compress_rows(M, K, b->tA[p], chi, b->tAc[p]);
        or_compress_rows(M, N, b->tC[p], chi, b->tCc[p]);
        or_compress_rows(M, N, b->tR[p], chi, b->tRc[p]);
        memcpy(b->tZc[p], b->tCc[p], (size_t)N * 16);
        or_matmul(1, K, N, b->Ec, b->tB[p], v);
        add_into(N, b->tZc[p], v);
        or_matmul(1, K, N, b->tAc[p], b->U, v);
        add_into(N, b->tZc[p], v);
        for (int64_t j = 0; j < N; j++) {
            st(b->tZc[p], j, ld(b->tZc[p], j) + (u128)delta[p] * ld(b->EUc, j));
            g_mults++;
            st(b->tDc[p], j, ld(b->tRc[p], j) - ld(b->tZc[p], j));
        }
        b->tag_mults[p] = g_mults - m0 + pub_mults + opt[p];
    }
    free(chi);
    free(v);
}

static void online_product(int mode, const or_desc *d, const uint64_t *delta, or_bufs *b);

/* The online phase.  A convolution opens U = Y - B on the input's shape (its
 * elements are what the parties broadcast) and then runs the product on the
 * im2col matrices of Y, B and their tags (Eq. (4)); im2col is linear, so these
 * are authenticated shares of the im2col matrices. */
void or_online(int mode, const or_desc *d, const uint64_t *delta, or_bufs *b) {
    or_set_kbits(d->kbits);
    if (d->conv_c <= 0) {
        online_product(mode, d, delta, b);
        return;
    }
    conv_validate(d);
    const int np = parties_of(d);
    const int64_t KN = d->K * d->N, nr = or_right_len(d);
    open_diff(np, nr, b->Y, b->B, b->U);
    or_bufs x = *b;
    uint64_t *tmp[4 * OR_MAX_PARTIES + 1];
    for (int i = 0; i < 4 * np + 1; i++) tmp[i] = alloc128(KN);
    for (int p = 0; p < np; p++) {
        or_im2col(d, b->Y[p], tmp[4 * p + 0]);
        or_im2col(d, b->tY[p], tmp[4 * p + 1]);
        or_im2col(d, b->B[p], tmp[4 * p + 2]);
        or_im2col(d, b->tB[p], tmp[4 * p + 3]);
        x.Y[p] = tmp[4 * p + 0];
        x.tY[p] = tmp[4 * p + 1];
        x.B[p] = tmp[4 * p + 2];
        x.tB[p] = tmp[4 * p + 3];
    }
    x.U = tmp[4 * np];
    or_desc dx = *d;
    dx.conv_c = 0;
    online_product(mode, &dx, delta, &x);
    for (int p = 0; p < np; p++) b->tag_mults[p] = x.tag_mults[p];
    for (int i = 0; i < 4 * np + 1; i++) free(tmp[i]);
}

static void online_product(int mode, const or_desc *d, const uint64_t *delta, or_bufs *b) {
    const int64_t K = d->K, N = d->N, rows = d->r1 - d->r0;
    const uint64_t seed = d->seed, lid = d->layer_id;
    const int np = parties_of(d);

    /* Fig. 7 online step 1: open E = X - A and U = Y - B. */
    open_diff(np, rows * K, b->X, b->A, b->E);
    open_diff(np, K * N, b->Y, b->B, b->U);

    /* Fig. 7 online step 2 and Eq. (2):
     *   [Z]_p = [C]_p + E*[B]_p + [A]_p*U, and the public term E*U is added by
     *   party 0 only (Fig. 2 step 3 / Fig. 7 step 4).  E*U is formed before D
     *   is opened (reading of Eq. (5) and the cost count of Sec. 3.4.3). */
    uint64_t *EU = alloc128(rows * N), *tmp = alloc128(rows * N);
    uint64_t m_eu = g_mults;
    or_matmul(rows, K, N, b->E, b->U, EU);
    const uint64_t eu_mults = g_mults - m_eu;
    for (int p = 0; p < np; p++) {
        memcpy(b->Z[p], b->C[p], (size_t)(rows * N) * 16);
        or_matmul(rows, K, N, b->E, b->B[p], tmp);
        add_into(rows * N, b->Z[p], tmp);
        or_matmul(rows, K, N, b->A[p], b->U, tmp);
        add_into(rows * N, b->Z[p], tmp);
    }
    add_into(rows * N, b->Z[0], EU);

    /* Open D = R - Z (Pi_OptMAC step 2 in COMPACT mode; Pi_Truncation step 1 in
     * SPDZ2k mode), kept as the full lift D~ mod 2^{k+s}. */
    open_diff(np, rows * N, b->R, b->Z, b->D);

    /* f > 0: truncation by the opened D (OptMAC&Trunc, Fig. 6, ExpandTrunc
     * steps 2-4, in CompactTag mode; Pi_Truncation, Fig. 3 online step 2, after
     * Pi_MatMul in SPDZ2k mode -- the same formulas).  D is reduced mod 2^k and
     * divided by 2^f as an integer in [0, 2^k):
     *   [Z^f]_p = [R^f]_p - D/2^f  (the public term by party 0 only),
     *   [tZ^f]_p = [tR^f]_p - [Delta]_p * D/2^f. */
    if (d->f > 0) {
        for (int64_t e = 0; e < rows * N; e++) {
            const uint64_t df = mod_k(ld(b->D, e)) >> d->f;
            for (int p = 0; p < np; p++) {
                st(b->Zf[p], e, ld(b->Rf[p], e) - (p == 0 ? (u128)df : (u128)0));
                st(b->tZf[p], e, ld(b->tRf[p], e) - (u128)delta[p] * df);
            }
        }
    }

    if (mode == OR_MODE_SPDZ2K) {
        /* Eq. (3): [tZ]_p = [tC]_p + E*[tB]_p + [tA]_p*U + [Delta]_p * (E*U);
         * the key term is added by every party (it is a share of Delta~ * EU).
         * Every party forms E*U itself, so its cost is charged to each. */
        for (int p = 0; p < np; p++) {
            uint64_t m0 = g_mults;
            memcpy(b->tZ[p], b->tC[p], (size_t)(rows * N) * 16);
            or_matmul(rows, K, N, b->E, b->tB[p], tmp);
            add_into(rows * N, b->tZ[p], tmp);
            or_matmul(rows, K, N, b->tA[p], b->U, tmp);
            add_into(rows * N, b->tZ[p], tmp);
            for (int64_t e = 0; e < rows * N; e++) {
                st(b->tZ[p], e, ld(b->tZ[p], e) + (u128)delta[p] * ld(EU, e));
                g_mults++;
            }
            b->tag_mults[p] = g_mults - m0 + eu_mults;
        }
    } else {
        /* Pi_OptMAC step 3: [tZ]_p = [tR]_p - [Delta]_p * D~. */
        uint64_t opt[OR_MAX_PARTIES];
        for (int p = 0; p < np; p++) {
            uint64_t m0 = g_mults;
            for (int64_t e = 0; e < rows * N; e++) {
                st(b->tZ[p], e, ld(b->tR[p], e) - (u128)delta[p] * ld(b->D, e));
                g_mults++;
            }
            opt[p] = g_mults - m0;
        }

        if (d->compress == 1) {
            compact_rows(d, delta, b, opt);
            free(EU);
            free(tmp);
            return;
        }
        /* Fig. 7 steps 5-6: public combiners chi in Z_{2^s}^{N x 1}, compress
         * tag(B), tag(C), U, tag(R) and D~ along N.  The public vectors U^c,
         * D~^c and E*U^c are formed by every party, so their cost is charged
         * to each. */
        uint64_t *chi = (uint64_t *)malloc((size_t)(N > 0 ? N : 1) * 8);
        if (!chi) abort();
        draw_chi(seed, stream_of(lid, OR_P_CHI), 0, N, chi);
        uint64_t m_pub = g_mults;
        or_compress(K, N, b->U, chi, b->Uc);
        or_compress(rows, N, b->D, chi, b->Dc);
        /* Eq. (5) / Fig. 7 step 7, with the key on the public term:
         *   [tZ^c]_p = [tC^c]_p + E*[tB^c]_p + [tA]_p*U^c + [Delta]_p * (E*U^c)
         *   [tD^c]_p = [tR^c]_p - [tZ^c]_p */
        or_matmul(rows, K, 1, b->E, b->Uc, b->EUc);
        const uint64_t pub_mults = g_mults - m_pub;
        uint64_t *v = alloc128(rows);
        for (int p = 0; p < np; p++) {
            uint64_t m0 = g_mults;
            or_compress(K, N, b->tB[p], chi, b->tBc[p]);
            or_compress(rows, N, b->tC[p], chi, b->tCc[p]);
            or_compress(rows, N, b->tR[p], chi, b->tRc[p]);
            memcpy(b->tZc[p], b->tCc[p], (size_t)rows * 16);
            or_matmul(rows, K, 1, b->E, b->tBc[p], v);
            add_into(rows, b->tZc[p], v);
            or_matmul(rows, K, 1, b->tA[p], b->Uc, v);
            add_into(rows, b->tZc[p], v);
            for (int64_t i = 0; i < rows; i++) {
                st(b->tZc[p], i, ld(b->tZc[p], i) + (u128)delta[p] * ld(b->EUc, i));
                g_mults++;
                st(b->tDc[p], i, ld(b->tRc[p], i) - ld(b->tZc[p], i));
            }
            b->tag_mults[p] = g_mults - m0 + pub_mults + opt[p];
        }
        free(chi);
        free(v);
    }
    free(EU);
    free(tmp);
}

/* ------------------------------------------------------------------ */
/* verification (what the GPU library calls mac_check)                  */

/* per-party tag shares of W = P - Q by linearity: [tW]_p = [tP]_p - [tQ]_p */
static void tag_diff(int64_t n, const uint64_t *tP, const uint64_t *tQ, uint64_t *out) {
    for (int64_t e = 0; e < n; e++) st(out, e, ld(tP, e) - ld(tQ, e));
}

void or_check(int mode, const or_desc *d, const uint64_t *delta, or_bufs *b) {
    or_set_kbits(d->kbits);
    const int np = parties_of(d);
    const int64_t M = d->M, K = d->K, N = d->N, r0 = d->r0, rows = d->r1 - d->r0;
    const uint64_t seed = d->seed, lid = d->layer_id;
    /* U is checked on the elements that were opened: K x N, or the input's shape */
    const int64_t nr = or_right_len(d);
    int64_t big = rows * K > nr ? rows * K : nr;
    if (rows * N > big) big = rows * N;
    uint64_t *tW = alloc128(big);
    uint64_t *chi = (uint64_t *)malloc((size_t)(big > M ? big : M) * 8);
    if (!chi) abort();
    (void)M;

    /* Fig. 7 verification step 1: Pi_BatchRec tag check of E and of U, one
     * public combiner per element (Fig. 1 tag-check step 1). */
    draw_chi(seed, stream_of(lid, OR_P_CHI_E), (uint64_t)(r0 * K), rows * K, chi);
    for (int p = 0; p < np; p++) {
        tag_diff(rows * K, b->tX[p], b->tA[p], tW);
        or_batchrec_cs(rows * K, b->E, tW, chi, delta[p], b->cs[0][p]);
    }
    draw_chi(seed, stream_of(lid, OR_P_CHI_U), 0, nr, chi);
    for (int p = 0; p < np; p++) {
        tag_diff(nr, b->tY[p], b->tB[p], tW);
        or_batchrec_cs(nr, b->U, tW, chi, delta[p], b->cs[1][p]);
    }

    if (mode == OR_MODE_SPDZ2K) {
        /* Pi_Truncation verification: Pi_BatchRec tag check of D = R - Z,
         * [tD]_p = [tR]_p - [tZ]_p. */
        draw_chi(seed, stream_of(lid, OR_P_CHI_D), (uint64_t)(r0 * N), rows * N, chi);
        for (int p = 0; p < np; p++) {
            tag_diff(rows * N, b->tR[p], b->tZ[p], tW);
            or_batchrec_cs(rows * N, b->D, tW, chi, delta[p], b->cs[2][p]);
        }
    } else {
        /* Fig. 7 verification steps 2-5: chihat in Z_{2^s}^{L x 1}, L the
         * length of D~^c (M when compressing along N, N when along M). */
        const int64_t first = d->compress == 1 ? 0 : r0, len = d->compress == 1 ? N : rows;
        uint64_t *ch = (uint64_t *)malloc((size_t)(len > 0 ? len : 1) * 8);
        if (!ch) abort();
        draw_chi(seed, stream_of(lid, OR_P_CHIHAT), (uint64_t)first, len, ch);
        for (int p = 0; p < np; p++) or_compact_cs(len, b->Dc, b->tDc[p], ch, delta[p], b->cs[2][p]);
        free(ch);
    }
    free(tW);
    free(chi);
}
