/*
 * compacttag.h -- C ABI of libcompacttag, the MI355X (gfx950) library for the
 * linear-layer hot path of actively secure MPC over Z_{2^64} (two parties by
 * default)
 * (CompactTag, arXiv 2311.04406).
 *
 * Setting (Sec. 2.4 of the paper): values live in Z_{2^k}, k = 64; value and
 * tag shares live in Z_{2^{k+s}} = Z_{2^128}, s = 64; the MAC key shares
 * [Delta]_p live in Z_{2^s}.  The parties p = 0 .. n-1 (n = 2 by default, up
 * to CT_MAX_PARTIES; the paper's appendix on scaling with parties) are
 * simulated in one process on one GPU; every "broadcast and reconstruct" of
 * the paper is an on-device sum of all parties' shares.
 *
 * Conventions shared by every entry point
 *   - Ring elements of Z_{2^128} are ct_u128 {lo, hi}: value = lo + 2^64 * hi.
 *   - Every matrix is row-major and contiguous; X is M x K, Y is K x N,
 *     Z = X * Y is M x N (the paper's T1 x T2, T2 x T3 and T1 x T3).
 *   - Every ct_u128 pointer in ct_layer_bufs is a DEVICE pointer, 16-byte
 *     aligned, allocated and owned by the caller; the library never frees
 *     caller memory and never allocates on the hot path (ct_tag_linear,
 *     ct_mac_check_device).  Buffers of different layers must not overlap.
 *   - Work is enqueued on the stream given in ct_params (NULL = the null
 *     stream) and is asynchronous unless stated otherwise.  A context is
 *     single-stream and not thread-safe; several contexts may coexist.
 *   - Errors are returned as ct_status; nothing is thrown across the ABI.
 *     CT_EINVAL: a null or misaligned pointer, M, K or N < 1, (k, s) not (64, 64) or (32, 32),
 *     f or in_bits outside [0, 63], n < 1 or more layers than the context
 *     was sized for.
 *     CT_EDEVICE: a HIP error (text in ct_last_error).  CT_ABORT is not a
 *     library error: it is the protocol's abort when a MAC check fails.
 */
#ifndef COMPACTTAG_H
#define COMPACTTAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint64_t lo, hi;
} ct_u128;

typedef enum { CT_OK = 0, CT_EINVAL = 1, CT_ENOMEM = 2, CT_EDEVICE = 3, CT_ABORT = 4 } ct_status;

/* CT_MODE_SPDZ2K: per-element tags of Eq. (3) (Pi_MatMul, Fig. 2), with D = R - Z
 *                 opened and batch-checked as in Pi_Truncation (Fig. 3).
 * CT_MODE_COMPACT: optimistic tag (Pi_OptMAC) verified through the compact tag
 *                 of Eq. (5) (Pi_CompactMatMul, Fig. 7). */
typedef enum { CT_MODE_SPDZ2K = 0, CT_MODE_COMPACT = 1 } ct_mode;

typedef struct ct_ctx ct_ctx;

/* Most parties a context simulates; every per-party array below has this many
 * slots, of which the first ct_params.parties are used. */
#define CT_MAX_PARTIES 5

typedef struct {
    int device;           /* HIP device ordinal */
    uint64_t key_seed;    /* seeds the key shares [Delta]_0, [Delta]_1 */
    int k_bits, s_bits;   /* the parameter set of Sec. 4.1: k = s = 64 (values in Z_{2^64}, shares,
                             tags and check values in Z_{2^128}, 16-byte elements) or k = s = 32
                             (values in Z_{2^32}, shares and tags in Z_{2^64}, 8-byte elements
                             uint64_t, key shares and combiners in Z_{2^32}) */
    void *hip_stream;     /* hipStream_t the context enqueues on; NULL = null stream */
    int max_layers;       /* largest n accepted by one call; <= 0 means 256 */
    int parties;          /* parties simulated, 2 .. CT_MAX_PARTIES; 0 means 2.  More than two
                             parties: plain products only (conv_c = 0), compressed along N, and
                             no request server */
} ct_params;

typedef struct {
    int64_t M, K, N;      /* X: M x K, Y: K x N */
    int32_t f;            /* fractional bits truncated after the product, 0..63.  f > 0:
                             truncation by the opened D (OptMAC&Trunc, Fig. 6, in
                             CT_MODE_COMPACT; Pi_Truncation, Fig. 3, in CT_MODE_SPDZ2K):
                             [Z^f]_p = [R^f]_p - (D mod 2^k) / 2^f (party 0 subtracts the
                             public term), [tZ^f]_p = [tR^f]_p - [Delta]_p (D mod 2^k) / 2^f,
                             written to Zf, tZf; the dealer adds the truncated mask
                             R^f = (R mod 2^k) / 2^f (Rf, tRf).  Z, tZ, D are still written. */
    int32_t in_bits;      /* dealer inputs: 0 = uniform in Z_{2^64}; 1..63 = signed in_bits-bit
                             integers in two's complement (a stand-in for fixed-point data) */
    uint64_t seed;        /* per-layer seed of the dealer and of the public combiners */
    uint64_t layer_id;    /* < 2^48; names the layer's generator streams */
    int32_t compress;     /* CT_MODE_COMPACT: the dimension Pi_Compress (Fig. 4) combines,
                             CT_COMPRESS_N, CT_COMPRESS_M or CT_COMPRESS_AUTO; ignored in
                             CT_MODE_SPDZ2K */
    int32_t reserved;     /* must be 0 */
    /* Convolution (Eq. (4)) with the im2col matrix left implicit: conv_c > 0
     * makes Y the im2col matrix of a conv_c x conv_h x conv_w input for a
     * conv_k x conv_k kernel, stride conv_stride, zero padding conv_pad (row
     * k = (c conv_k + dy) conv_k + dx, column n = y Wo + x holds input element
     * (c, y stride + dy - pad, x stride + dx - pad), 0 in the padding).  Then
     * K = conv_c conv_k^2 and N = Ho Wo with Ho = (conv_h + 2 pad - conv_k) /
     * stride + 1 (Wo alike) are required, N > CT_SKINNY_N, and Y, tY, B, tB, U
     * hold CT_RIGHT_LEN = conv_c conv_h conv_w elements: the input, the mask B
     * of the input's shape (the triple is C = A im2col(B)) and the opened
     * U = Y - B, which the parties broadcast and the check of U covers.
     * conv_c = 0: a plain product (the other conv fields must be 0). */
    int32_t conv_c, conv_h, conv_w, conv_k, conv_stride, conv_pad;
} ct_layer_desc;

/* Elements of Y, tY, B, tB and U of a layer. */
#define CT_RIGHT_LEN(d) ((d).conv_c > 0 ? (int64_t)(d).conv_c * (d).conv_h * (d).conv_w : (d).K * (d).N)

/* The compressed dimension of the compact tag.  The notation of Sec. 2.2
 * leaves it open; the operation count of Sec. 3.4.3 is 4MN + 2KN + 3MK + M
 * along N and 4MN + 2KM + 3KN + N along M, so AUTO takes M exactly when
 * M > N (e.g. a classifier layer at batch 1).
 *   CT_COMPRESS_N: W^c = W chi with chi of length N (the columns are combined);
 *     the compact tag, Eq. (5), is a vector of length M, chihat has length M.
 *   CT_COMPRESS_M: W^c = chi^T W with chi of length M; Eq. (5) multiplied by
 *     chi^T from the left, [tZ^c]_p = [tC^c]_p + E^c [tB]_p + [tA^c]_p U +
 *     [Delta]_p E^c U with E^c = chi^T E, [tA^c]_p = chi^T [tA]_p (length K);
 *     the compact tag has length N, chihat has length N.
 * chi and chihat are drawn from the same streams in both cases. */
#define CT_COMPRESS_N 0
#define CT_COMPRESS_M 1
#define CT_COMPRESS_AUTO 2
#define CT_COMPRESS_ALONG_M(M, N, c) ((c) == CT_COMPRESS_M || ((c) == CT_COMPRESS_AUTO && (M) > (N)))

/* Per-layer device buffers.  [v]_p / [t v]_p are party p's value / tag share
 * (slots p < parties are used; the others are ignored).
 * Every element is one element of Z_{2^{k+s}}: a ct_u128 for k = s = 64, a
 * uint64_t (the pointer still typed ct_u128 *) for k = s = 32.  Element
 * counts (CT_WORK_LEN, CT_CVEC_LEN) are the same for both. */
typedef struct {
    ct_u128 *X[CT_MAX_PARTIES], *tX[CT_MAX_PARTIES], *A[CT_MAX_PARTIES], *tA[CT_MAX_PARTIES];                   /* M x K */
    ct_u128 *Y[CT_MAX_PARTIES], *tY[CT_MAX_PARTIES], *B[CT_MAX_PARTIES], *tB[CT_MAX_PARTIES];                   /* K x N (convolution: the input's shape) */
    ct_u128 *C[CT_MAX_PARTIES], *tC[CT_MAX_PARTIES], *R[CT_MAX_PARTIES], *tR[CT_MAX_PARTIES], *Z[CT_MAX_PARTIES], *tZ[CT_MAX_PARTIES];    /* M x N; Z, tZ are outputs */
    ct_u128 *E, *U, *D;  /* opened public values E = X - A (M x K), U = Y - B (K x N, or the input's shape),
                            D = R - Z (M x N); outputs of ct_tag_linear */
    ct_u128 *cvec;       /* compact-tag vectors, CT_CVEC_LEN_FOR(M, K, N, compress) elements
                            (n parties: CT_CVEC_LEN_NP), layout below;
                            written by ct_tag_linear in CT_MODE_COMPACT, unused otherwise */
    ct_u128 *work;       /* caller-owned workspace of CT_WORK_LEN(M, K, N) elements (n parties:
                            CT_WORK_LEN_NP; NULL allowed when that is 0); contents are undefined
                            after a call */
    ct_u128 *Rf[CT_MAX_PARTIES], *tRf[CT_MAX_PARTIES];  /* M x N, f > 0 only: truncated mask (written by the dealer) */
    ct_u128 *Zf[CT_MAX_PARTIES], *tZf[CT_MAX_PARTIES];  /* M x N, f > 0 only: truncated output shares and tags */
} ct_layer_bufs;

/* Layers with N <= CT_SKINNY_N form their output products in the pass that
 * opens E (bandwidth-bound, no workspace); wider layers use the matrix cores
 * and a workspace holding the folded left operands A_0 + E and, in SPDZ2k
 * mode, [tA]_p + [Delta]_p E (three M x K arrays), then the operands of the
 * products converted to 8-bit digit tiles (five left operands of
 * 64 x 32-element tiles over M x K and five right ones over N x K, 2048
 * elements per tile).  The matrix-core path needs K < 2^21 and N < 2^22. */
#define CT_SKINNY_N 8
#define CT_TILES_(D, K) ((((D) + 63) / 64) * (((K) + 31) / 32))
#define CT_WORK_LEN(M, K, N) CT_WORK_LEN_NP(M, K, N, 2)
/* With n parties: the folded operands A_0 + E and (SPDZ2k) [tA]_p + [Delta]_p E
 * (n + 1 arrays of M x K) and 2n + 1 packed operands on each side. */
#define CT_WORK_LEN_NP(M, K, N, n) \
    ((N) > CT_SKINNY_N ? ((n) + 1) * (M) * (K) + (2 * (n) + 1) * 2048 * (CT_TILES_(M, K) + CT_TILES_(N, K)) : 0)

/* cvec layout (element offsets), compressing along N:
 *   U^c [K] | tB^c_0 [K] | tB^c_1 [K] | D^c [M] | (E U^c) [M] | tC^c_0 [M] | tC^c_1 [M] |
 *   tR^c_0 [M] | tR^c_1 [M] | tZ^c_0 [M] | tZ^c_1 [M] | tD^c_0 [M] | tD^c_1 [M];
 * compressing along M, the same with U^c, tB^c_p replaced by E^c, tA^c_p and
 * every [M] by [N] (D^c = chi^T D, (E^c U), tC^c_p = chi^T tC_p, ...). */
#define CT_CVEC_LEN(M, K) (3 * (K) + 10 * (M))
/* n parties (compressing along N): U^c [K] | tB^c_p [K] for p < n | D^c [M] |
 * (E U^c) [M] | tC^c_p [M] | tR^c_p [M] | tZ^c_p [M] | tD^c_p [M], each per-party
 * group in party order; with n = 2 the layout above. */
#define CT_CVEC_LEN_NP(M, K, n) ((1 + (n)) * (K) + (2 + 4 * (n)) * (M))
#define CT_CVEC_LEN_FOR(M, K, N, c) (3 * (K) + 10 * (CT_COMPRESS_ALONG_M(M, N, c) ? (N) : (M)))

/* Check-value shares of one layer: cs[W][p] for W = 0 (E), 1 (U), 2 (D) and
 * parties p < n (the other slots are 0).  accept = 1 iff sum_p cs[W][p] = 0
 * mod 2^{k+s} for all three W.  reserved is 0, except 1 when a persistent
 * launch's barrier wait ran out (accept is then 0; see ct_set_launch). */
typedef struct {
    ct_u128 cs[3][CT_MAX_PARTIES];
    int32_t accept;
    int32_t reserved;
} ct_check_result;

/* Creates a context on params->device: samples the key shares
 * [Delta]_p = draw(key_seed, stream (0xFFFF << 16) | (0x40 + p), 0) (F_MAC
 * Initialize, Appendix A) and keeps them resident, and allocates the
 * context's own fixed-size device scratch (descriptor tables, check
 * accumulators).  *out receives the context; free it with ct_destroy. */
ct_status ct_create(ct_ctx **out, const ct_params *params);

/* Releases the context and its scratch after synchronizing its stream. */
ct_status ct_destroy(ct_ctx *ctx);

/* Copies the key shares of the context's n parties to host memory out[0 .. n-1]. */
ct_status ct_key_shares(const ct_ctx *ctx, uint64_t out[CT_MAX_PARTIES]);

/* Dealer (preprocessing of Fig. 7 and F_MAC Auth, Appendix A), for n layers:
 * Beaver matrix triple A (M x K), B (K x N), C = A*B mod 2^128 (M x N) and the
 * mask R (M x N), all uniform in Z_{2^128}, and, if with_inputs != 0, inputs
 * X (M x K) and Y (K x N) uniform in Z_{2^64} (or signed in_bits-bit values;
 * upper limb zero).  For f > 0 also the truncated mask of Figs. 3 and 6,
 * R^f = (R mod 2^64) / 2^f, its upper limb a fresh uniform draw.  Every object
 * is authenticated: [v]_0 and [tv]_0 are fresh draws, [v]_1 = v~ - [v]_0 and
 * [tv]_1 = Delta~ * v~ - [tv]_0 with Delta~ = [Delta]_0 + [Delta]_1 taken as an
 * integer.  Writes X, tX, Y, tY (if with_inputs), A, tA, B, tB, C, tC, R, tR
 * (and Rf, tRf) of both parties.  Asynchronous. */
ct_status ct_gen_triple_tags(ct_ctx *ctx, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                             int with_inputs);

/* Online phase of n linear layers (Fig. 7 online steps 1-7 for
 * CT_MODE_COMPACT; Fig. 2 with Eqs. (2)-(3) plus the opening of D for
 * CT_MODE_SPDZ2K).  Reads X, tX, A, tA, Y, tY, B, tB, C, tC, R, tR; writes
 * E, U, D, Z, tZ (and cvec in CT_MODE_COMPACT).  Party 0 adds the public term
 * E*U to its value share; every party adds its key share times a public term
 * to its tag share.  Layers with f > 0 also read Rf, tRf and write the
 * truncated output Zf, tZf (see ct_layer_desc.f).  Asynchronous; allocates
 * nothing. */
ct_status ct_tag_linear(ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n);

/* Verification of n layers, results left in device memory: writes n
 * ct_check_result records to the device array out_dev (the accept field is
 * computed on the device).  Pi_BatchRec tag check (Fig. 1) of E and U in both
 * modes and of D = R - Z in CT_MODE_SPDZ2K (Pi_Truncation, Fig. 3); the
 * compact check of D (Fig. 7 verification steps 2-6) in CT_MODE_COMPACT.  All
 * check values are reduced mod 2^128.  The public combiners are drawn from the
 * layer's generator streams, so a layer's results do not depend on the other
 * layers in the call.  Asynchronous; allocates nothing.  Reads the arrays
 * again, independently of how ct_tag_linear produced them. */
ct_status ct_mac_check_device(ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B,
                              int n, ct_check_result *out_dev);

/* The online phase and the verification of n layers in one pass over the
 * data: the same outputs as ct_tag_linear followed by ct_mac_check_device and
 * the same n check records in out_dev, but each check sum is accumulated by
 * the kernel that opens the checked value (E and U from the input shares, D
 * after the products), so no share array is read twice.  This is the
 * amortised verification of many products in one shot.  Asynchronous;
 * allocates nothing.  A batch that mixes layers with N > CT_SKINNY_N and
 * layers with N <= CT_SKINNY_N runs the former on a second stream of the
 * context, forked from the context stream after its earlier work and joined
 * back before its later work, so the two groups overlap; every check record
 * still lands at its layer's position in out_dev.  With per-kernel timing
 * enabled (ct_set_timing) the whole batch runs on the context stream. */
ct_status ct_tag_linear_check(ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                              ct_check_result *out_dev);

/* Bytes of the static workspace of ct_tag_linear_check_static: 256 MiB per GPU. */
#define CT_STATIC_WORK_BYTES (256LL << 20)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: exactly
 * ct_tag_linear_check (same outputs, same check records in out_dev), except
 * that the workspace of the layers with N > CT_SKINNY_N comes from a static
 * array of CT_STATIC_WORK_BYTES that the library holds on each GPU for the
 * life of the process; B[l].work is ignored.  The layers' workspaces
 * (CT_WORK_LEN_NP(M, K, N, parties) elements each, at 256-byte boundaries)
 * must fit in it together: otherwise CT_EINVAL with the sizes in
 * ct_last_error, and nothing runs.  Allocates no device memory (no hipMalloc,
 * hipFree or other allocating call); the caller still passes every input and
 * output buffer.  Every call on one GPU
 * uses the same array and leaves undefined contents in it (every byte a call
 * reads there it has written first), so calls that overlap on one GPU --
 * from contexts on different streams, or from several threads -- race and
 * must be serialized by the caller.  Asynchronous. */
ct_status ct_tag_linear_check_static(ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B,
                                     int n, ct_check_result *out_dev);

/* As ct_mac_check_device, then waits for the stream and copies the n results
 * to host memory out.  Returns CT_ABORT if any layer fails its check (out is
 * still filled, so the caller can see which check value failed). */
ct_status ct_mac_check(ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                       ct_check_result *out);

/* Optional per-kernel timing, for profiling: while enabled, every kernel the
 * context launches is bracketed by a pair of HIP events recorded on the
 * context stream.  The first enable creates the context's event pool (2048
 * pairs); when the pool is full the stream is synchronized and the pairs are
 * folded into per-stage totals.  Not for use under graph capture. */
ct_status ct_set_timing(ct_ctx *ctx, int enable);

/* Whether ct_tag_linear_check and plans created afterwards run the two
 * layer groups of a mixed batch on two streams (enable != 0, the default) or
 * the whole batch on the context stream (0: every kernel then runs alone,
 * as a per-kernel profile needs).  Results are the same either way. */
ct_status ct_set_overlap(ct_ctx *ctx, int enable);

/* How ct_tag_linear_check (and ct_tag_linear_check_static, and plans created
 * afterwards) launch the online phase of a batch of two parties (Sec. 3.3:
 * the layers of a batch are tagged and verified together).
 *   CT_LAUNCH_STAGED (the default): one multi-layer kernel per stage, each
 *     at the occupancy its registers allow.
 *   CT_LAUNCH_PERSISTENT: the whole online phase and its fused check in one
 *     launch of one 256-thread workgroup per compute unit, which walks the
 *     stages over all layers and meets at a grid barrier between stages;
 *     every stage then runs at the product kernel's occupancy (four
 *     wavefronts per compute unit).  It applies to calls (and plans) that
 *     carry the fused check and whose layers are all matrix-core layers
 *     (N > CT_SKINNY_N) that are neither convolutions nor compressed along
 *     M; other calls, and the request server's batches, take the staged
 *     kernels.  The results are the same bit for bit.  A barrier wait is
 *     bounded (ct_set_launch_wait, 2 s by default); if one runs out, every
 *     layer's check record reports accept = 0 and reserved = 1.  The launch
 *     needs every workgroup resident at once: do not run other work on the
 *     device beside it.
 * Returns CT_EINVAL for another mode. */
#define CT_LAUNCH_STAGED 0
#define CT_LAUNCH_PERSISTENT 1
ct_status ct_set_launch(ct_ctx *ctx, int mode);

/* Bound of each grid-barrier wait of the persistent launch, in ticks of the
 * device's 100 MHz wall clock (CT_LAUNCH_WAIT_DEFAULT: 2 s).  A wait that
 * runs out sets the launch's run-out flag, every later wait of the launch
 * ends at once, and every layer's check record reports accept = 0 and
 * reserved = 1 (the outputs are then not to be used).  A tiny bound lets a
 * caller exercise that report.  Applies to launches enqueued afterwards
 * (a plan keeps the bound it was captured with). */
#define CT_LAUNCH_WAIT_DEFAULT 200000000ull
ct_status ct_set_launch_wait(ct_ctx *ctx, uint64_t ticks);

typedef struct {
    char name[24];        /* kernel stage, e.g. "ring_gemm", "check_batch" */
    double total_ms;      /* summed event-measured duration */
    int64_t launches;     /* number of launches summed */
} ct_stage_time;

/* Synchronizes the stream and returns, per kernel stage launched since the
 * previous call, the summed duration and launch count (at most max records;
 * *count receives the number of stages), then resets the totals. */
ct_status ct_stage_times(ct_ctx *ctx, ct_stage_time *out, int max, int *count);

/* Product kernel and workgroup tile shape (ct_tuning.tile).  Both kernels
 * compute the same exact products (identical results); a workgroup of four
 * wavefronts owns 64 x 64 outputs, or 128 x 64 with two 32 x 32 tiles per
 * wavefront, which only the k = s = 32 set has registers for (with
 * k = s = 64 the 128 x 64 shapes run as 64 x 64).
 *   CT_TILE_AUTO: register-streamed; 128 x 64 for k = s = 32 when the launch
 *     has at least two such tiles per compute unit, else 64 x 64.
 *   CT_TILE_LDS_*: operand digit tiles copied global -> LDS, one K slice
 *     ahead, fragments read from LDS (a workgroup barrier per K slice).
 *   CT_TILE_REGS_*: every wavefront loads its digit fragments from global
 *     memory into registers one K slice ahead; no LDS, no barriers.
 *   CT_TILE_REGS_FIT: register-streamed, one 32 x 32 tile per wavefront, the
 *     workgroup tile chosen per layer from 64 x 64, 32 x 128 and 128 x 32 as
 *     the one with the fewest padded outputs (64 x 64 on ties). */
#define CT_TILE_AUTO 0
#define CT_TILE_LDS_64x64 1
#define CT_TILE_LDS_128x64 2
#define CT_TILE_REGS_64x64 3
#define CT_TILE_REGS_128x64 4
#define CT_TILE_REGS_FIT 5

/* Launch configuration of the matrix-core products. */
typedef struct {
    int32_t group_m;       /* output row tiles per group of the tile order (>= 1) */
    int32_t xcd_remap;     /* 0: tiles in list order (blocks go round-robin over the 8 XCDs);
                              1: each XCD gets a contiguous range of the list; G >= 2: groups of
                              G consecutive tiles go round-robin over the XCDs, so the tiles of a
                              group share one XCD's L2 */
    int32_t split_target;  /* K slices of 32 per tile; 0 = as many tiles as fill the GPU twice */
    int32_t tile;          /* CT_TILE_*: product kernel and workgroup tile shape */
    double gemm_ms;        /* ct_autotune: measured duration of the products per call, with the copy
                              of the constant terms into the outputs of K-split products */
} ct_tuning;

/* Autotuner: runs the online phase of this batch of layers (outputs written
 * as by ct_tag_linear) once per candidate launch configuration, times the
 * matrix-core products and the copy of the constant terms that K-split
 * products need first, with HIP events (reps timed runs after one warm-up
 * each), and keeps the fastest for this shape class -- the protocol and the
 * rounded-up binary logarithms of M, K, N of every matrix-core layer.  The
 * candidates are a coordinate descent from the current configuration: the
 * tile shape and kernel (CT_TILE_LDS_64x64, CT_TILE_REGS_64x64,
 * CT_TILE_REGS_FIT, and for k = s = 32 also the 128 x 64 shapes), then
 * split_target in 0, 16, 32, 64, 128, xcd_remap in 0, 1, 4, 8, 16 and
 * group_m in 1, 2, 4, 8, 16, 64, each under the best so far, then the tile
 * shape again.  Later calls of the same class use the choice.  Synchronizes;
 * allocates the timing event pool if timing was never enabled; the stage
 * times of ct_stage_times are left as they were.  best (may be NULL)
 * receives the choice. */
ct_status ct_autotune(ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n, int reps,
                      ct_tuning *best);

/* The configuration a call with these layers would use (gemm_ms = -1). */
ct_status ct_get_tuning(const ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, int n, ct_tuning *out);

/* Sets the configuration of shape classes never tuned and forgets all tuned
 * ones. */
ct_status ct_set_tuning(ct_ctx *ctx, const ct_tuning *t);

/* ---- Captured plans: one graph launch per step (HIP graphs) ----
 *
 * A plan records the online phase of a fixed batch of layers (exactly as
 * ct_tag_linear, or as ct_tag_linear_check when out_dev is not NULL) once
 * into a HIP graph: its descriptor tables are uploaded into device memory the
 * plan owns before the capture, so the graph holds kernel nodes only.  The
 * layer buffers, out_dev and the launch configuration (ct_autotune's choice
 * for the batch at creation time) are bound at creation; every launch
 * recomputes all outputs from the current contents of the input buffers.
 * A mixed batch is captured as two branches of the graph, as
 * ct_tag_linear_check runs it on two streams.  Creating a plan allocates;
 * launching one does not. */
typedef struct ct_plan ct_plan;

/* Validates as ct_tag_linear_check does (out_dev may be NULL: no
 * verification), captures and instantiates the graph.  Synchronizes. */
ct_status ct_plan_create(ct_ctx *ctx, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                         ct_check_result *out_dev, ct_plan **out);

/* Launches the plan's graph on the context stream.  Asynchronous. */
ct_status ct_plan_launch(ct_plan *plan);

/* Waits for the plan's launches and frees it. */
ct_status ct_plan_destroy(ct_plan *plan);

/* ---- Request server: continuous batching over one device arena ----
 *
 * Serves a stream of tag-generation and verification requests of mixed
 * layer shapes on one GPU.  A TAG request names a layer (shape, seed,
 * layer_id): the server admits it when its footprint fits in the arena,
 * draws its inputs and triple there with the dealer, and runs the online
 * phase (as ct_gen_triple_tags with inputs, then ct_tag_linear, in the
 * server's protocol).  The layer then stays resident -- shares, tags, key
 * shares' products, public values -- for later checks.  A CHECK request
 * names a shape: it runs the MAC checks (as ct_mac_check_device) on the most
 * recent complete resident layer of that shape, and runs as a TAG if there
 * is none.  Admission is first come, first served by scheduled arrival time;
 * requests that have arrived while others are on the device form the next
 * batch as soon as one of the server's slots (HIP streams) is free, so work
 * of successive batches overlaps on the device.  Complete layers are
 * evicted least recently used first when a TAG does not fit.  A layer's
 * results do not depend on the other requests of its batch (the check
 * combiners are keyed by the layer's seed and layer_id).
 *
 * The server runs a worker thread that owns the context from ct_server_create
 * to ct_server_destroy: the context must not be used by any other call in
 * that time.  The server allocates its slots' tables at creation and nothing
 * afterwards; all layer memory comes from the caller's arena. */
typedef struct ct_server ct_server;

/* CT_REQ_PREP: the preprocessing of a layer ahead of its TAG request (the
 * offline phase, Sec. 3.5; inputs and triple are input-independent material
 * here, drawn by the dealer): admitted by footprint like a TAG, it runs only
 * the dealer and leaves the layer resident as prepared.  A later TAG request
 * for the same layer (M, K, N, seed, layer_id) then runs only the online
 * phase on it -- waiting, first come first served, if the preparation is
 * still on the device.  The TAG's results are the same as without the PREP.
 * A prepared layer no TAG has taken may be evicted (after every complete
 * layer), and its TAG then deals the layer itself. */
typedef enum { CT_REQ_TAG = 0, CT_REQ_CHECK = 1, CT_REQ_PREP = 2 } ct_req_kind;

typedef struct {
    void *arena;          /* device memory for resident layers and workspaces (caller-owned,
                             256-byte aligned, not used by the caller while the server lives) */
    size_t arena_bytes;
    int32_t slots;        /* batches in flight at once, one HIP stream each: 1..8 */
    int32_t max_batch;    /* most requests in one batch: 1..256 */
    int32_t mode;         /* ct_mode of the TAG requests and of the checks */
    int32_t reserved;
} ct_server_params;

typedef struct {
    int64_t id;           /* the caller's request id, unique per server: a request whose id is that of
                             a layer still resident (a TAG not yet evicted, or a CHECK that ran as
                             one) completes with CT_EINVAL and does not run */
    int32_t kind;         /* ct_req_kind */
    int32_t reserved;
    ct_layer_desc layer;  /* TAG: the layer (f must be 0); CHECK: only M, K, N are used */
    double arrival_us;    /* scheduled arrival on the server clock (ct_server_now_us); the request is
                             not admitted earlier, and its latency counts from this time */
} ct_request;

typedef struct {
    int64_t id;
    int32_t kind;         /* as executed */
    int32_t status;       /* CT_OK; CT_ABORT: the check rejected; CT_ENOMEM: the layer does not fit in
                             the arena at all; CT_EINVAL: the id names a resident layer (not run);
                             CT_EDEVICE: a HIP error (ct_server_last_error) */
    int64_t layer;        /* id of the TAG request whose layer this request wrote or checked (-1 if none) */
    double arrival_us, admit_us, done_us;  /* server clock; done_us: completion seen by the worker */
    int32_t batch_size, slot;
    ct_check_result result;  /* CHECK: the layer's check values */
} ct_completion;

typedef struct {
    int64_t submitted, completed, rejected, converted, evictions, batches, max_batch, resident_layers;
    uint64_t arena_bytes, arena_peak, arena_used;
    int64_t duplicates;   /* requests refused (CT_EINVAL) because their id named a resident layer */
    int64_t prepared;     /* PREP requests admitted */
    int64_t online_only;  /* TAG requests that ran the online phase only, on a prepared layer */
} ct_server_counts;

/* Creates the server's slots and starts its worker thread. */
ct_status ct_server_create(ct_ctx *ctx, const ct_server_params *params, ct_server **out);

/* Microseconds since the server was created (the clock of arrival_us). */
double ct_server_now_us(const ct_server *server);

/* Queues n requests (validated first: on CT_EINVAL none is queued).  A
 * request's layer is a plain product (conv_c = 0) with f = 0, K < 2^21 and
 * N < 2^22; any compressed dimension. */
ct_status ct_server_submit(ct_server *server, const ct_request *reqs, int n);

/* Moves up to max completions, in completion order, into out; *count
 * receives their number.  Non-blocking. */
ct_status ct_server_poll(ct_server *server, ct_completion *out, int max, int *count);

/* Waits until every submitted request has completed (CT_EDEVICE after
 * timeout_s seconds). */
ct_status ct_server_drain(ct_server *server, double timeout_s);

/* Descriptor and device buffers of the complete resident layer written by
 * TAG request id (work = NULL).  The buffers stay valid until the server
 * evicts the layer, which only an admission can do: read them while no
 * request is pending. */
ct_status ct_server_layer(ct_server *server, int64_t id, ct_layer_desc *desc, ct_layer_bufs *bufs);

ct_status ct_server_stats(ct_server *server, ct_server_counts *out);

/* Stops admitting, waits for the batches in flight, stops the worker and
 * frees the slots (queued requests that were never admitted are dropped). */
ct_status ct_server_destroy(ct_server *server);

const char *ct_server_last_error(ct_server *server);

/* Text of the last error on this context ("" if none). */
const char *ct_last_error(const ct_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* COMPACTTAG_H */
