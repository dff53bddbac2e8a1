// ct_internal.h -- library-internal types shared by the host side of
// libcompacttag and its HIP kernels.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "compacttag.h"

namespace ct {

// Element of Z_{2^128}: value = lo + 2^64 hi (same layout as ct_u128).
struct u128 {
    uint64_t lo, hi;
};
// An element of Z_{2^64}: shares and tags of the k = s = 32 parameter set.
struct r64 {
    uint64_t v;
};

// Generator stream purposes; stream = (layer_id << 16) | purpose.
enum Purpose : uint32_t {
    P_LIFT_X = 0x01, P_LIFT_Y = 0x02, P_LIFT_A = 0x03, P_LIFT_B = 0x04, P_LIFT_R = 0x05,
    P_LIFT_RF = 0x06,  // upper limb of the lift of the truncated mask R^f
    P_VSH = 0x10,  // + object 1..7
    P_TSH = 0x20,  // + object 1..7
    P_CHI = 0x30, P_CHIHAT = 0x31, P_CHI_E = 0x32, P_CHI_U = 0x33, P_CHI_D = 0x34,
    P_KEY = 0x40,  // + party, on the global layer id 0xFFFF
};
enum Obj : int { OBJ_X = 1, OBJ_Y = 2, OBJ_A = 3, OBJ_B = 4, OBJ_C = 5, OBJ_R = 6, OBJ_RF = 7 };
constexpr int NUM_OBJ = 7;
constexpr uint64_t GLOBAL_LAYER = 0xFFFF;

// Index of each generator key in LayerDev::key.
enum KeyIdx : int {
    K_LIFT_X = 0, K_LIFT_Y, K_LIFT_A, K_LIFT_B, K_LIFT_R, K_LIFT_RF,
    K_VSH_X, K_VSH_Y, K_VSH_A, K_VSH_B, K_VSH_C, K_VSH_R, K_VSH_RF,
    K_TSH_X, K_TSH_Y, K_TSH_A, K_TSH_B, K_TSH_C, K_TSH_R, K_TSH_RF,
    K_CHI, K_CHIHAT, K_CHI_E, K_CHI_U, K_CHI_D,
    K_COUNT
};

// Geometry of a convolution layer whose right operand is the implicit im2col
// matrix of a c x h x w input (Eq. (4)); on = 0 for a plain product.
struct ConvGeom {
    int32_t on, c, h, w, k, s, p, wo;
};

// Element of the input under entry (k, n) of the im2col matrix:
// k = (c k + dy) k + dx, n = y wo + x -> (c, y s + dy - p, x s + dx - p);
// -1 where that falls in the zero padding.  k < 2^21, n < 2^22.
__host__ __device__ inline int64_t conv_src(const ConvGeom &g, int32_t k, int32_t n) {
    const uint32_t kk = (uint32_t)(g.k * g.k);
    const uint32_t c = (uint32_t)k / kk, t = (uint32_t)k - c * kk;
    const uint32_t dy = t / (uint32_t)g.k, dx = t - dy * (uint32_t)g.k;
    const uint32_t y = (uint32_t)n / (uint32_t)g.wo, x = (uint32_t)n - y * (uint32_t)g.wo;
    const int32_t iy = (int32_t)(y * g.s + dy) - g.p, ix = (int32_t)(x * g.s + dx) - g.p;
    if (iy < 0 || iy >= g.h || ix < 0 || ix >= g.w) return -1;
    return ((int64_t)c * g.h + iy) * g.w + ix;
}
// Index of right-operand entry (k, n) in a layer's K x N-shaped or input-shaped buffers.
__host__ __device__ inline int64_t kn_src(const ConvGeom &g, int64_t N, int64_t k, int64_t n) {
    return g.on ? conv_src(g, (int32_t)k, (int32_t)n) : k * N + n;
}

// Per-layer descriptor as the kernels see it (device memory).
// The two-party kernels use slots 0 and 1 of the per-party arrays; the
// n-party kernels (np > 2) slots 0 .. np - 1.
constexpr int MAXP = CT_MAX_PARTIES;
struct LayerDev {
    int64_t M, K, N;
    uint64_t delta[MAXP];       // key shares
    uint64_t key[K_COUNT];      // SplitMix64 stream keys
    u128 *X[MAXP], *tX[MAXP], *A[MAXP], *tA[MAXP];
    u128 *Y[MAXP], *tY[MAXP], *B[MAXP], *tB[MAXP];
    u128 *C[MAXP], *tC[MAXP], *R[MAXP], *tR[MAXP], *Z[MAXP], *tZ[MAXP];
    u128 *E, *U, *D, *cvec;
    u128 *work;                 // caller workspace: A_0 + E | tA_p + Delta_p E for p < np (M x K each), then
                                // the packed operands
    u128 *acc;                  // check accumulators, ACC_PER_LAYER entries (context scratch)
    u128 *Rf[MAXP], *tRf[MAXP], *Zf[MAXP], *tZf[MAXP];  // f > 0: truncated mask and output (M x N)
    int32_t f, in_bits;         // truncated fractional bits; dealer input width (0: uniform)
    int32_t cm;                 // CompactTag compresses along M (W^c = chi^T W) instead of N
    int32_t np;                 // parties
    ConvGeom cv;                // convolution geometry (cv.on = 0: plain product)
    int64_t nr;                 // elements of Y, tY, B, tB, U: K N, or c h w of a convolution
    // share streams of parties 1 .. np - 2 (party 0 uses key[K_VSH_X + obj - 1] and
    // key[K_TSH_X + obj - 1]; the last party completes the sums)
    uint64_t vsh[MAXP - 2][NUM_OBJ], tsh[MAXP - 2][NUM_OBJ];
    // two-party matrix-core layers that are not convolutions: U is opened by
    // k_open_pack, which also writes the digit tiles of [B]_0, [B]_1 and U
    // (rp[0..2], in the workspace); k_open_u skips them
    int32_t fo;
    int32_t out_index;          // position of the layer's check record in the caller's result array
    u128 *rp[3];
};

// cvec offsets of n parties, compressing along N (see compacttag.h): U^c,
// tB^c_p (K each), then D^c, E U^c, tC^c_p, tR^c_p, tZ^c_p, tD^c_p (M each).
struct NpCvec {
    int64_t Uc, tBc, Dc, EUc, tCc, tRc, tZc, tDc, K, M;
    __host__ __device__ int64_t tb(int p) const { return tBc + p * K; }
    __host__ __device__ int64_t tc(int p) const { return tCc + p * M; }
    __host__ __device__ int64_t tr(int p) const { return tRc + p * M; }
    __host__ __device__ int64_t tz(int p) const { return tZc + p * M; }
    __host__ __device__ int64_t td(int p) const { return tDc + p * M; }
};
__host__ __device__ inline NpCvec np_cvec(int64_t M, int64_t K, int np) {
    NpCvec o;
    o.K = K; o.M = M;
    o.Uc = 0; o.tBc = K; o.Dc = (1 + np) * K; o.EUc = o.Dc + M;
    o.tCc = o.Dc + 2 * M; o.tRc = o.tCc + np * M; o.tZc = o.tRc + np * M; o.tDc = o.tZc + np * M;
    return o;
}

// Layers with N <= SKINNY_MAX_N take their output products on the VALU inside
// the pass that opens E (no MFMA tiles, no workspace).
constexpr int SKINNY_MAX_N = 8;

// Elements of one row of E per work item of the row pass (a multiple of 64,
// at least 1024): long rows are cut into several items, so that a layer
// with few rows still spreads over the whole GPU; segments double while the
// layer keeps at least 16384 items.  Each item ends in wavefront reductions
// and atomic additions of its row products, so short items cost: on the
// batched set (K from 32 to 4096) the pass took 1.22 ms with items of at
// least 256 elements, 0.87 ms with 512 and 0.77 ms with 1024.
__host__ __device__ inline int64_t row_seg(int64_t M, int64_t K) {
    int64_t s = 1024;
    while (s < 4096 && M * ((K + 2 * s - 1) / (2 * s)) >= 16384) s *= 2;
    return s;
}
__host__ __device__ inline int64_t row_items(int64_t M, int64_t K) {
    const int64_t s = row_seg(M, K);
    return M * ((K + s - 1) / s);
}

// Flags of the fused passes.
enum PassFlags : int {
    F_CHECK = 1,    // accumulate the MAC-check sums of the values the pass opens
    F_COMPACT = 2,  // CompactTag protocol (compression, compact tag)
    F_SPDZ = 4,     // SPDZ2k protocol (per-element tags by products)
};

// Check accumulators per layer.  Two parties: for W in (E, U, D) at 3 W:
// [sum chi*tW_0, sum chi*tW_1, sum chi*W].  n parties: at W (CT_MAX_PARTIES + 1):
// [sum chi*tW_p for p < n ..., sum chi*W at slot CT_MAX_PARTIES].
constexpr int ACC_W = CT_MAX_PARTIES + 1;
// The row passes add their check sums of E into copies of their
// accumulators held as 32-bit limbs in 64-bit cells (atomic_add_limbs), from
// element ACC_RP of the layer's accumulators on: workgroup b adds into copy
// b % RP_COPIES (two parties: 3 sums, 12 cells a copy) or b % NP_RP_COPIES
// (n parties: ACC_W sums, 4 ACC_W cells), so that concurrent workgroups add
// to different cells without waiting; k_finalize / k_np_finalize add the
// copies to the E sums.
constexpr int ACC_RP = 3 * ACC_W;
constexpr int RP_CELLS = 1536;  // 64-bit cells (768 elements of 16 bytes)
constexpr int RP_COPIES = RP_CELLS / 12;
constexpr int NP_RP_COPIES = RP_CELLS / (4 * ACC_W);
constexpr int ACC_PER_LAYER = 3 * ACC_W + RP_CELLS / 2;

// cvec offsets (elements), see compacttag.h.  Compressing along M the same
// offsets are taken with M replaced by N (cvec_off(N, K)), and the three
// K-long vectors hold E^c, [tA^c]_0, [tA^c]_1 in place of U^c, [tB^c]_p.
struct CvecOff {
    int64_t Uc, tBc0, tBc1, Dc, EUc, tCc0, tCc1, tRc0, tRc1, tZc0, tZc1, tDc0, tDc1;
};
__host__ __device__ inline CvecOff cvec_off(int64_t M, int64_t K) {
    CvecOff o;
    o.Uc = 0; o.tBc0 = K; o.tBc1 = 2 * K; o.Dc = 3 * K; o.EUc = 3 * K + M;
    o.tCc0 = 3 * K + 2 * M; o.tCc1 = 3 * K + 3 * M; o.tRc0 = 3 * K + 4 * M; o.tRc1 = 3 * K + 5 * M;
    o.tZc0 = 3 * K + 6 * M; o.tZc1 = 3 * K + 7 * M; o.tDc0 = 3 * K + 8 * M; o.tDc1 = 3 * K + 9 * M;
    return o;
}

// Length of the compressed M x N quantities (D^c, the compact tags): M when
// compressing along N, N when compressing along M.
__host__ __device__ inline int64_t cvec_rows(const LayerDev &L) { return L.cm ? L.N : L.M; }

// Variant of the row pass a layer takes: 0 for matrix-core layers, else the
// smallest of 1, 2, 4, 8 that holds N.  Each variant is its own kernel so the
// register budget (and occupancy) of one does not limit the others.
__host__ __device__ inline int row_variant(int64_t N) {
    return N > SKINNY_MAX_N ? 0 : (N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : SKINNY_MAX_N)));
}

// With more than two parties, the fused row pass serves matrix-core layers and
// layers with N <= 2 (its per-party row products fit in registers); layers
// with 2 < N <= SKINNY_MAX_N take the separate opening, product and compact
// passes.
__host__ __device__ inline bool np_fused_row(int64_t N) { return N > SKINNY_MAX_N || N <= 2; }

// Row pass of a layer compressed along M: lanes own columns; a wavefront
// takes a strip of cm_cw(N) * 64 columns over CM_RB rows and keeps the column
// sums chi_m E_mk, chi_m [tA]_p,mk in registers until its rows are done
// (narrower strips for skinny layers, whose row products take registers too).
constexpr int CM_RB = 32;
__host__ __device__ constexpr int cm_cw_variant(int ns) { return ns == 0 || ns == 1 ? 4 : (ns == 2 ? 2 : 1); }
__host__ __device__ inline int cm_cw(int64_t N) {
    return cm_cw_variant(N > 8 ? 0 : (N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8))));
}
// Bit of the row-pass variant set: 1 << v for k_row_pass<v>, 1 << (VARIANT_CM + v)
// for k_row_pass_cm<v> (v = 0, 1, 2, 4, 8).
constexpr int VARIANT_CM = 16;
__host__ __device__ inline int64_t cm_strips(int64_t K, int cw) { return (K + 64 * cw - 1) / (64 * cw); }
__host__ __device__ inline int64_t cm_items(int64_t M, int64_t K, int64_t N) {
    return cm_strips(K, cm_cw(N)) * ((M + CM_RB - 1) / CM_RB);
}

// Column sweep (sums down the columns of a rows x N matrix): wavefront items
// of rb groups of 64 / G rows (N <= 32, G = pow2ceil(N); one atomic per column
// per item) or of 64 columns x rb rows (one per lane).  rb = col_sweep_rb keeps
// the atomic additions per column near 256 at most (same-address atomics
// serialize) without starving the sweep of wavefronts.
__host__ __device__ inline int64_t col_sweep_group(int64_t N) {
    int64_t g = 1;
    while (g < N) g <<= 1;
    return g;
}
__host__ __device__ inline int64_t col_sweep_rb(int64_t rows, int64_t N) {
    if (N <= 32) {
        const int64_t per = (64 / col_sweep_group(N)) * 256, rb = (rows + per - 1) / per;
        return rb < 1 ? 1 : rb;
    }
    const int64_t rb = (rows + 255) / 256;
    return rb < 4 ? 4 : rb;
}
__host__ __device__ inline int64_t col_sweep_items(int64_t rows, int64_t N) {
    const int64_t rb = col_sweep_rb(rows, N);
    if (N <= 32) {
        const int64_t per = (64 / col_sweep_group(N)) * rb;
        return (rows + per - 1) / per;
    }
    return ((N + 63) / 64) * ((rows + rb - 1) / rb);
}

// Operands of the matrix-core products are converted once into "digit
// tiles": for an operand with major dimension D (rows of a left operand,
// columns of a right operand) and contraction length K, tile (t, ks) covers
// major indices [64 t, 64 t + 64) and k in [32 ks, 32 ks + 32); it occupies
// TILE_ELEMS elements at ((t * KT) + ks) * TILE_ELEMS and holds one plane of
// signed 8-bit digits per digit of an element (plane d = digit d; 16 planes,
// 32 KB, for Z_{2^128}; 8 planes, 16 KB, for Z_{2^64}) of 64 x 32 bytes, in the
// byte order of the GEMM's LDS stage.  Out-of-range entries are zero.
constexpr int TILE_ELEMS = 2048;

inline int64_t packed_elems(int64_t major, int64_t K) { return ((major + 63) / 64) * ((K + 31) / 32) * TILE_ELEMS; }

// Workspace of a layer with N > SKINNY_MAX_N (element offsets): the folded
// left operands written by the row pass, then the digit tiles of every
// operand of the matrix-core products.
struct WorkOff {
    int64_t AE0, tAE0, tAE1;                  // u128, M x K each
    int64_t Ep, AE0p, A1p, tAE0p, tAE1p;      // packed left operands
    int64_t B0p, B1p, Up, tB0p, tB1p;         // packed right operands
    int64_t total;
};
inline WorkOff work_off(int64_t M, int64_t K, int64_t N) {
    WorkOff o;
    const int64_t mk = M * K, pl = packed_elems(M, K), pr = packed_elems(N, K);
    o.AE0 = 0; o.tAE0 = mk; o.tAE1 = 2 * mk;
    o.Ep = 3 * mk; o.AE0p = o.Ep + pl; o.A1p = o.Ep + 2 * pl; o.tAE0p = o.Ep + 3 * pl; o.tAE1p = o.Ep + 4 * pl;
    o.B0p = o.Ep + 5 * pl; o.B1p = o.B0p + pr; o.Up = o.B0p + 2 * pr; o.tB0p = o.B0p + 3 * pr;
    o.tB1p = o.B0p + 4 * pr;
    o.total = o.B0p + 5 * pr;
    return o;
}

// One packing job: src (row-major rows x cols) -> dst digit tiles.
// side 0: left operand (major = row, k = column); side 1: right operand
// (major = column, k = row).
struct PackJob {
    const u128 *src;
    u128 *dst;
    int32_t rows, cols, side, majt, kt, tile_begin, tiles, pad;
    ConvGeom cv;  // right operand read as the implicit im2col matrix of src (cv.on)
};

// One ring GEMM problem over packed operands (one party's product of a layer;
// the products of a layer form a group whose tiles are interleaved):
//   out (+)= base + L1 * R1 + L2 * R2     (all mod 2^128)
// Lp1, Lp2: packed M x K left operands; Rp1, Rp2: packed K x N right
// operands; out, base: M x N row-major.  Lp2 == nullptr: single segment.
// accumulate != 0: out already holds base and partial sums of K splits are
// added atomically.
struct GemmProb {
    const u128 *Lp1, *Lp2, *Rp1, *Rp2, *base;
    u128 *out;
    int32_t M, N, K, accumulate;
    int32_t tiles_m, tiles_n, splits, steps_per_split;  // steps are 32-wide K slices
    int32_t kt, nsteps, tile_begin, tiles;  // tile_begin, tiles: of the problem's layer group
    int32_t group_m;  // tile order: column sweeps over groups of group_m row tiles
    int32_t gfirst;   // index of the first problem of the layer group (problems of one layer
    int32_t gsize;    //   share M, N, K and splits and are interleaved in the tile order)
    int32_t mt;       // 32 x 32 output tiles per wavefront, stacked in M (the same for every
                      // problem of a launch): workgroup tiles of 64 mt x 64 outputs
    int32_t wshape;   // WaveShape of the workgroup tile (register-streamed kernel, mt = 1)
};

// Arrangement of the four wavefronts of a register-streamed workgroup at one
// 32 x 32 output tile each: 2 x 2 (64 x 64 outputs), 1 x 4 (32 x 128) or
// 4 x 1 (128 x 32).  The wavefronts load their fragments independently, so
// any arrangement reads the same packed operand tiles; the narrow ones pad a
// product's M (or N) to 32 instead of 64.
enum WaveShape : int { WS_64x64 = 0, WS_32x128 = 1, WS_128x32 = 2 };

// Product kernels: operand tiles staged through LDS, or fragments streamed
// from global memory into registers.
enum GemmKernel : int { GEMM_LDS = 0, GEMM_REGS = 1 };

// Launch configuration of the matrix-core products (chosen by ct_autotune).
struct GemmTuning {
    int32_t group_m;       // row tiles per group of the tile order (1 = row-major order)
    int32_t xcd_remap;     // 0: identity; 1: contiguous range per XCD; G >= 2: groups of G tiles per XCD
    int32_t split_target;  // K slices per tile; 0 = enough tiles for two rounds over the CUs
    int32_t tile;          // CT_TILE_*: kernel and workgroup tile (0 = by the launch's size)
};

// Unpacked product for the dealer's layers with N <= SKINNY_MAX_N:
// out = L * R (L: M x K, R: K x N, row-major).
struct SkinnyProb {
    const u128 *L, *R;
    u128 *out;
    int32_t M, N, K, pad;
};

// The two-party online phase of a batch as one persistent launch
// (k_online_persist): the stages' tables as the staged kernels take them, and
// the launch's counters, sync[0 .. 12), all 0 at the launch: sync[0] counts
// workgroup arrivals at the grid barriers, sync[1] is set when a barrier wait
// ran out (after wait_ticks of the 100 MHz wall clock), sync[4 + x] hands
// out the product tiles of XCD x.
struct PersistArgs {
    const LayerDev *Ls;
    const PackJob *jobs;
    const GemmProb *probs;
    ct_check_result *out;
    uint32_t *sync;
    uint64_t wait_ticks;
    int32_t n, flags, zero_what, njobs, pack_tiles, nprobs, total_tiles, xcd_remap, any_accum, mt;
};

// ---- launchers (defined in the .hip files) ----
// eb: bytes per ring element, 16 (k = s = 64) or 8 (k = s = 32).
hipError_t launch_pack(int eb, const PackJob *jobs_dev, int njobs, int total_tiles, hipStream_t st);
// kernel: GEMM_LDS (operand tiles staged through LDS, k_ring_gemm) or
// GEMM_REGS (fragments streamed into registers, k_ring_gemm_rs)
hipError_t launch_gemm(int eb, const GemmProb *probs_dev, int nprobs, int total_tiles, int xcd_remap, int mt,
                       int kernel, hipStream_t st);
// The persistent launch: `wgs` workgroups of 256 threads, one per compute
// unit (all must be resident at once: the stages meet at grid barriers).
hipError_t launch_online_persist(int eb, const PersistArgs &a, int wgs, hipStream_t st);
hipError_t launch_skinny(int eb, const SkinnyProb *probs_dev, int nprobs, int max_rows, hipStream_t st);

hipError_t launch_fill_zero(int eb, u128 *p, int64_t n, hipStream_t st);
hipError_t launch_deal_lift(int eb, const LayerDev *L, int n, int64_t max_elems, hipStream_t st);
hipError_t launch_deal_auth(int eb, const LayerDev *L, int n, int obj, int64_t max_elems, hipStream_t st);
hipError_t launch_zero_acc(int eb, const LayerDev *L, int n, int what, int64_t max_elems, hipStream_t st);
hipError_t launch_open_u(int eb, const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st);
hipError_t launch_open_pack(int eb, const LayerDev *L, int n, int flags, int max_tiles, hipStream_t st);
// variants: bit v (bit VARIANT_CM + v) set if some layer takes row-pass variant v (0, 1, 2, 4, 8)
// (of the pass of layers compressed along M)
hipError_t launch_row_pass(int eb, const LayerDev *L, int n, int flags, int64_t max_items, int variants, hipStream_t st);
hipError_t launch_post(int eb, const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st);
hipError_t launch_compact_final(int eb, const LayerDev *L, int n, int flags, hipStream_t st);
hipError_t launch_col_tag(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st);
hipError_t launch_conv_compress(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st);

// n-party path (ct_parties.hip)
hipError_t launch_np_lift(int eb, const LayerDev *L, int n, int64_t max_elems, hipStream_t st);
hipError_t launch_np_auth(int eb, const LayerDev *L, int n, int obj_mask, int64_t max_elems, hipStream_t st);
hipError_t launch_np_zero(int eb, const LayerDev *L, int n, int what, int64_t max_elems, hipStream_t st);
hipError_t launch_np_open(int eb, const LayerDev *L, int n, int which, int flags, int64_t max_elems, hipStream_t st);
hipError_t launch_prob_base(int eb, const GemmProb *probs, int nprobs, int64_t max_mn, hipStream_t st);
hipError_t launch_np_skinny(int eb, const LayerDev *L, int n, int flags, int64_t max_items, hipStream_t st);
hipError_t launch_np_post(int eb, const LayerDev *L, int n, int flags, int64_t max_elems, hipStream_t st);
hipError_t launch_np_compress(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st);
// variants: bit v set if some fused layer takes row-pass variant v (0, 1, 2)
hipError_t launch_np_row_pass(int eb, int np, const LayerDev *L, int n, int flags, int64_t max_items, int variants,
                              hipStream_t st);
hipError_t launch_np_gemv(int eb, const LayerDev *L, int n, int64_t max_items, hipStream_t st);
hipError_t launch_np_compact_final(int eb, const LayerDev *L, int n, int flags, hipStream_t st);
hipError_t launch_np_check_batch(int eb, const LayerDev *L, int n, int which_mask, int64_t max_elems, hipStream_t st);
hipError_t launch_np_check_compact(int eb, const LayerDev *L, int n, hipStream_t st);
hipError_t launch_np_finalize(int eb, const LayerDev *L, int n, ct_check_result *out, hipStream_t st);
hipError_t launch_check_batch(int eb, const LayerDev *L, int n, int which, int64_t max_elems, hipStream_t st);
hipError_t launch_check_compact(int eb, const LayerDev *L, int n, hipStream_t st);
hipError_t launch_finalize(int eb, const LayerDev *L, int n, ct_check_result *out, hipStream_t st);

// Number of wavefront work items of a row sweep over an R x N matrix (the
// grid of the sweeping kernels is sized from it).
inline int64_t sweep_items(int64_t rows, int64_t N) {
    if (N <= 64) {
        int64_t g = 1;
        while (g < N) g <<= 1;
        const int64_t rpw = 64 / g;
        return (rows + rpw - 1) / rpw;
    }
    return rows * ((N + 511) / 512);
}

// Workgroup items of k_conv_compress: (input channel, segment of 512 output
// positions) of a convolution with c input channels and N output positions.
inline int64_t conv_compress_items(int64_t c, int64_t N) { return c * ((N + 511) / 512); }

}  // namespace ct
