/*
 * ct_oracle.h -- interface of the CPU oracle (test infrastructure only).
 *
 * This header belongs to oracle/ and to nothing else: the GPU library has its
 * own header and shares no code, constant or helper with this one.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * the oracle.
 *
 * Ring elements of Z_{2^{k+s}} are stored as two little-endian uint64 limbs
 * (lo, hi); with k = s = 32 the high limb is always zero.  Matrices are
 * row-major.  A "rows" range [r0, r1) restricts every
 * M-indexed quantity to those rows of the M dimension; with r0 = 0 and r1 = M
 * the oracle runs the whole procedure.  K x N quantities are always complete.
 */
#ifndef CT_ORACLE_H
#define CT_ORACLE_H
#include <stdint.h>

#define OR_MODE_SPDZ2K 0
#define OR_MODE_COMPACT 1

/* Parties of one computation: 2 to OR_MAX_PARTIES (Appendix "CompactTag
 * scales with parties"); every per-party array below has this many slots, of
 * which the first `parties` are used. */
#define OR_MAX_PARTIES 5

/* Purposes of the counter-based generator streams; stream = (layer_id << 16) | purpose. */
#define OR_P_LIFT_X 0x01
#define OR_P_LIFT_Y 0x02
#define OR_P_LIFT_A 0x03
#define OR_P_LIFT_B 0x04
#define OR_P_LIFT_R 0x05
#define OR_P_LIFT_RF 0x06 /* upper limb of the lift of the truncated mask R^f */
#define OR_P_VSH 0x10 /* + object index 1..7 (X, Y, A, B, C, R, R^f) */
#define OR_P_TSH 0x20 /* + object index 1..7 */
#define OR_P_CHI 0x30
#define OR_P_CHIHAT 0x31
#define OR_P_CHI_E 0x32
#define OR_P_CHI_U 0x33
#define OR_P_CHI_D 0x34
#define OR_P_KEY 0x40 /* + party, on the global layer id 0xFFFF */
#define OR_GLOBAL_LAYER 0xFFFFULL

typedef struct {
    int64_t M, K, N;          /* X is M x K, Y is K x N, Z is M x N */
    uint64_t seed, layer_id;  /* per-layer randomness */
    int64_t r0, r1;           /* rows of the M dimension that are computed */
    int64_t f;                /* fractional bits truncated from the product (0: no truncation) */
    int64_t in_bits;          /* 0: inputs uniform in Z_{2^k}; 1..k-1: signed in_bits-bit inputs */
    int64_t kbits;            /* k = s: 64 (shares in Z_{2^128}) or 32 (shares in Z_{2^64}); 0 means 64 */
    int64_t compress;         /* dimension CompactTag compresses: 0 = N (combine the columns),
                                 1 = M (combine the rows; needs r0 = 0, r1 = M) */
    /* Convolution (Eq. (4)): conv_c > 0 makes Y the im2col matrix of a
     * conv_c x conv_h x conv_w input for a conv_k x conv_k kernel with stride
     * conv_stride and zero padding conv_pad; then K = conv_c conv_k^2, N = Ho Wo
     * (Ho = (conv_h + 2 conv_pad - conv_k) / conv_stride + 1, Wo alike), and the
     * buffers Y, tY, B, tB, U hold conv_c x conv_h x conv_w elements: the input,
     * its mask and the opened U of that shape.  conv_c = 0: a plain product. */
    int64_t conv_c, conv_h, conv_w, conv_k, conv_stride, conv_pad;
    int64_t parties;          /* 2..OR_MAX_PARTIES; 0 means 2 */
} or_desc;

/* Every pointer is a caller-owned array of (lo, hi) uint64 pairs. */
typedef struct {
    /* rows x K */
    uint64_t *X[OR_MAX_PARTIES], *tX[OR_MAX_PARTIES], *A[OR_MAX_PARTIES], *tA[OR_MAX_PARTIES], *E;
    /* K x N */
    uint64_t *Y[OR_MAX_PARTIES], *tY[OR_MAX_PARTIES], *B[OR_MAX_PARTIES], *tB[OR_MAX_PARTIES], *U;
    /* rows x N */
    uint64_t *C[OR_MAX_PARTIES], *tC[OR_MAX_PARTIES], *R[OR_MAX_PARTIES], *tR[OR_MAX_PARTIES];
    uint64_t *Z[OR_MAX_PARTIES], *tZ[OR_MAX_PARTIES], *D;
    /* compact-tag vectors, compress = 0: K entries */
    uint64_t *Uc, *tBc[OR_MAX_PARTIES];
    /* compact-tag vectors, compress = 0: rows entries (W^c = W chi);
     * compress = 1: N entries (W^c = chi^T W, and EUc holds E^c U) */
    uint64_t *Dc, *EUc;
    uint64_t *tCc[OR_MAX_PARTIES], *tRc[OR_MAX_PARTIES], *tZc[OR_MAX_PARTIES], *tDc[OR_MAX_PARTIES];
    /* compact-tag vectors, compress = 1: K entries, E^c = chi^T E and [tA^c]_p = chi^T [tA]_p */
    uint64_t *Ec, *tAc[OR_MAX_PARTIES];
    /* f > 0, rows x N: truncated mask R^f (dealt) and truncated output Z^f */
    uint64_t *Rf[OR_MAX_PARTIES], *tRf[OR_MAX_PARTIES], *Zf[OR_MAX_PARTIES], *tZf[OR_MAX_PARTIES];
    /* check-value shares cs[W][party][limb], W in (E, U, D) */
    uint64_t cs[3][OR_MAX_PARTIES][2];
    /* local multiplications spent on tags, per party */
    uint64_t tag_mults[OR_MAX_PARTIES];
} or_bufs;

uint64_t or_mix64(uint64_t z);
uint64_t or_stream_key(uint64_t seed, uint64_t stream);
uint64_t or_draw(uint64_t seed, uint64_t stream, uint64_t i);
void or_draw_many(uint64_t seed, uint64_t stream, uint64_t first, int64_t n, uint64_t *out);

void or_key_shares(uint64_t key_seed, uint64_t delta[2]);
void or_key_shares_k(uint64_t key_seed, int64_t kbits, uint64_t delta[2]);
/* key shares of parties 0..parties-1 */
void or_key_shares_n(uint64_t key_seed, int64_t kbits, int64_t parties, uint64_t *delta);
/* Ring width of the building blocks below (k = s = kbits); or_deal,
 * or_online and or_check set it from their descriptor. */
void or_set_kbits(int64_t kbits);
/* delta holds the key shares of the descriptor's parties */
void or_deal(const or_desc *d, const uint64_t *delta, int with_inputs, or_bufs *b);
void or_online(int mode, const or_desc *d, const uint64_t *delta, or_bufs *b);
void or_check(int mode, const or_desc *d, const uint64_t *delta, or_bufs *b);

/* Elements of the right operand's buffers: conv_c conv_h conv_w, or K N. */
int64_t or_right_len(const or_desc *d);
/* Eq. (4): out (K x N) = im2col of in (conv_c x conv_h x conv_w). */
void or_im2col(const or_desc *d, const uint64_t *in, uint64_t *out);

/* building blocks, exposed so tests can feed chosen combiners */
void or_matmul(int64_t M, int64_t K, int64_t N, const uint64_t *P, const uint64_t *Q, uint64_t *out);
void or_compress(int64_t rows, int64_t N, const uint64_t *Mx, const uint64_t *chi, uint64_t *out);
void or_compress_rows(int64_t rows, int64_t N, const uint64_t *Mx, const uint64_t *chi, uint64_t *out);
void or_batchrec_cs(int64_t n, const uint64_t *W, const uint64_t *tW, const uint64_t *chi,
                    uint64_t delta_p, uint64_t out[2]);
void or_compact_cs(int64_t rows, const uint64_t *Dc, const uint64_t *tDc, const uint64_t *chihat,
                   uint64_t delta_p, uint64_t out[2]);

#endif
