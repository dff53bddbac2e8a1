// ct_api.hip -- host side of the libcompacttag C ABI (see compacttag.h).
//
// A call validates its layers, writes one LayerDev record per layer (sizes,
// key shares, generator stream keys, buffer pointers) and the GEMM problem
// list into pinned staging memory, uploads them with one asynchronous copy on
// the context stream, and enqueues the kernels of the requested phase.  The
// staging area is reused only after the previous upload has completed (an
// event), so a call never allocates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "compacttag.h"
#include "ct_host.h"
#include "ct_internal.h"

using namespace ct;

static const char *kStageNames[ST_COUNT] = {
    "deal_lift", "fill_zero", "deal_auth", "deal_skinny", "zero_acc", "open_u", "row_pass", "pack",
    "copy_base", "ring_gemm", "post", "compact_final", "check_batch", "check_compact", "finalize", "col_tag",
    "conv_compress", "np_open", "np_skinny", "np_compress", "np_gemv", "open_pack", "persistent"};
constexpr int EV_POOL = 2048;

struct ct_plan {
    ct_ctx *ctx = nullptr;
    Lane lane, side;  // side: the matrix-core layers of a mixed batch (forked in the graph)
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// The workspace of ct_tag_linear_check_static: one file-scope array that each
// GPU holds for the life of the process.  Host code never passes the name
// itself to a kernel (on the host it is only a stand-in): ct_create takes the
// device address with hipGetSymbolAddress once per device, with that device
// current, and every use goes through that address.
static __device__ __align__(256) uint8_t scratch[CT_STATIC_WORK_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};  // device address of `scratch` per device

// Device address of this device's `scratch` (the device must be current).
hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

// ---- SplitMix64 (Steele, Lea, Flood 2014), host side ----
uint64_t hmix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
uint64_t hkey(uint64_t seed, uint64_t layer_id, uint64_t purpose) {
    return hmix(seed ^ hmix((layer_id << 16) | purpose));
}
uint64_t hdraw(uint64_t key, uint64_t i) { return hmix(key + (i + 1) * 0x9E3779B97F4A7C15ull); }

ct_status hip_fail(ct_ctx *c, hipError_t e, const char *where) {
    return fail(c, CT_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}
#define HIPCHK(ctx, expr)                                          \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);   \
    } while (0)

// Folds the recorded event pairs into the per-stage totals (synchronizes).
hipError_t fold_timing(ct_ctx *c) {
    if (c->ev_used == 0) return hipSuccess;
    hipError_t e = hipStreamSynchronize(c->main.stream);
    if (e != hipSuccess) return e;
    for (int i = 0; i < c->ev_used; i++) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, c->ev_start[i], c->ev_end[i]);
        if (e != hipSuccess) return e;
        c->stage_ms[c->ev_stage[i]] += ms;
        c->stage_n[c->ev_stage[i]] += 1;
    }
    c->ev_used = 0;
    return hipSuccess;
}

// Runs a launcher on lane ln; with timing on (main lane only), brackets it
// with an event pair on the lane's stream.
#define LAUNCH(ctx, ln, stage, expr)                                                     \
    do {                                                                                 \
        const bool timed_ = (ctx)->timing && (ln).timed;                                 \
        if (timed_) {                                                                    \
            if ((ctx)->ev_used == EV_POOL) HIPCHK(ctx, fold_timing(ctx));                \
            HIPCHK(ctx, hipEventRecord((ctx)->ev_start[(ctx)->ev_used], (ln).stream));   \
        }                                                                                \
        HIPCHK(ctx, expr);                                                               \
        if (timed_) {                                                                    \
            HIPCHK(ctx, hipEventRecord((ctx)->ev_end[(ctx)->ev_used], (ln).stream));     \
            (ctx)->ev_stage[(ctx)->ev_used++] = (stage);                                 \
        }                                                                                \
    } while (0)

bool aligned16(const void *p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

enum Need : unsigned {
    NEED_INPUTS = 1,   // X, tX, Y, tY
    NEED_TRIPLE = 2,   // A, tA, B, tB, C, tC, R, tR
    NEED_OUT = 4,      // Z, tZ, E, U, D
    NEED_CVEC = 8,
    NEED_WORK = 16,    // workspace of layers with N > SKINNY_MAX_N
};

ct_status validate(ct_ctx *c, int max_layers, const ct_layer_desc *L, const ct_layer_bufs *B, int n, unsigned need) {
    if (!c) return CT_EINVAL;
    if (!L || !B) return fail(c, CT_EINVAL, "null layer or buffer array");
    if (n < 1 || n > max_layers)
        return fail(c, CT_EINVAL, "n must be in [1, max_layers] (" + std::to_string(max_layers) + ")");
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        const std::string at = "layer " + std::to_string(l) + ": ";
        if (d.M < 1 || d.K < 1 || d.N < 1) return fail(c, CT_EINVAL, at + "M, K, N must be >= 1");
        if (d.M >= (1LL << 31) || d.K >= (1LL << 31) || d.N >= (1LL << 31))
            return fail(c, CT_EINVAL, at + "M, K, N must be < 2^31");
        if (d.f < 0 || d.f > 63) return fail(c, CT_EINVAL, at + "f must be in [0, 63]");
        if (d.in_bits < 0 || d.in_bits > 63) return fail(c, CT_EINVAL, at + "in_bits must be in [0, 63]");
        if (d.layer_id >= (1ULL << 48)) return fail(c, CT_EINVAL, at + "layer_id must be < 2^48");
        if (d.compress < CT_COMPRESS_N || d.compress > CT_COMPRESS_AUTO || d.reserved != 0)
            return fail(c, CT_EINVAL, at + "compress must be CT_COMPRESS_N, _M or _AUTO and reserved 0");
        if (d.conv_c < 0) return fail(c, CT_EINVAL, at + "conv_c must be >= 0");
        if (d.conv_c == 0 && (d.conv_h | d.conv_w | d.conv_k | d.conv_stride | d.conv_pad) != 0)
            return fail(c, CT_EINVAL, at + "convolution fields must be 0 when conv_c is 0");
        if (d.conv_c > 0) {
            const int64_t kk = d.conv_k, st = d.conv_stride, pd = d.conv_pad;
            if (kk < 1 || st < 1 || pd < 0 || pd >= kk || d.conv_h < 1 || d.conv_w < 1 ||
                d.conv_h + 2 * pd < kk || d.conv_w + 2 * pd < kk)
                return fail(c, CT_EINVAL, at + "invalid convolution geometry");
            const int64_t ho = (d.conv_h + 2 * pd - kk) / st + 1, wo = (d.conv_w + 2 * pd - kk) / st + 1;
            if (d.K != (int64_t)d.conv_c * kk * kk || d.N != ho * wo)
                return fail(c, CT_EINVAL, at + "K and N must be conv_c conv_k^2 and the output size Ho Wo");
            if (d.N <= SKINNY_MAX_N)
                return fail(c, CT_EINVAL, at + "convolution layers need N > CT_SKINNY_N");
        }
        const ct_layer_bufs &b = B[l];
        auto chk = [&](const ct_u128 *p, const char *name) -> bool {
            if (!aligned16(p)) {
                c->err = at + "buffer " + name + " is null or not 16-byte aligned";
                return false;
            }
            return true;
        };
        if (c->np > 2 && (d.conv_c != 0 || CT_COMPRESS_ALONG_M(d.M, d.N, d.compress)))
            return fail(c, CT_EINVAL, at + "more than two parties: plain products compressed along N only");
        for (int p = 0; p < c->np; p++) {
            if (need & NEED_INPUTS)
                if (!chk(b.X[p], "X") || !chk(b.tX[p], "tX") || !chk(b.Y[p], "Y") || !chk(b.tY[p], "tY"))
                    return CT_EINVAL;
            if (need & NEED_TRIPLE)
                if (!chk(b.A[p], "A") || !chk(b.tA[p], "tA") || !chk(b.B[p], "B") || !chk(b.tB[p], "tB") ||
                    !chk(b.C[p], "C") || !chk(b.tC[p], "tC") || !chk(b.R[p], "R") || !chk(b.tR[p], "tR"))
                    return CT_EINVAL;
            if (need & NEED_OUT)
                if (!chk(b.Z[p], "Z") || !chk(b.tZ[p], "tZ")) return CT_EINVAL;
            if (d.f > 0 && (need & NEED_TRIPLE))
                if (!chk(b.Rf[p], "Rf") || !chk(b.tRf[p], "tRf")) return CT_EINVAL;
            if (d.f > 0 && (need & NEED_OUT))
                if (!chk(b.Zf[p], "Zf") || !chk(b.tZf[p], "tZf")) return CT_EINVAL;
        }
        if (need & NEED_OUT)
            if (!chk(b.E, "E") || !chk(b.U, "U") || !chk(b.D, "D")) return CT_EINVAL;
        if (need & NEED_CVEC)
            if (!chk(b.cvec, "cvec")) return CT_EINVAL;
        if ((need & NEED_WORK) && d.N > SKINNY_MAX_N) {
            if (!chk(b.work, "work")) return CT_EINVAL;
            if (d.K >= (1LL << 21) || d.N >= (1LL << 22))
                return fail(c, CT_EINVAL, at + "matrix-core path needs K < 2^21 and N < 2^22");
        }
    }
    return CT_OK;
}

void fill_layer(const ct_ctx *c, u128 *acc, const ct_layer_desc &d, const ct_layer_bufs &b, int l, LayerDev &o) {
    std::memset(&o, 0, sizeof(o));
    o.M = d.M;
    o.K = d.K;
    o.N = d.N;
    o.np = c->np;
    for (int q = 0; q < c->np; q++) o.delta[q] = c->delta[q];
    const uint64_t s = d.seed, id = d.layer_id;
    o.key[K_LIFT_X] = hkey(s, id, P_LIFT_X);
    o.key[K_LIFT_Y] = hkey(s, id, P_LIFT_Y);
    o.key[K_LIFT_A] = hkey(s, id, P_LIFT_A);
    o.key[K_LIFT_B] = hkey(s, id, P_LIFT_B);
    o.key[K_LIFT_R] = hkey(s, id, P_LIFT_R);
    o.key[K_LIFT_RF] = hkey(s, id, P_LIFT_RF);
    for (int obj = 1; obj <= NUM_OBJ; obj++) {
        o.key[K_VSH_X + obj - 1] = hkey(s, id, P_VSH + obj);
        o.key[K_TSH_X + obj - 1] = hkey(s, id, P_TSH + obj);
        // parties 1 .. np - 2: the streams of purpose + 256 p
        for (int q = 1; q + 1 < c->np; q++) {
            o.vsh[q - 1][obj - 1] = hkey(s, id, P_VSH + obj + 256 * q);
            o.tsh[q - 1][obj - 1] = hkey(s, id, P_TSH + obj + 256 * q);
        }
    }
    o.key[K_CHI] = hkey(s, id, P_CHI);
    o.key[K_CHIHAT] = hkey(s, id, P_CHIHAT);
    o.key[K_CHI_E] = hkey(s, id, P_CHI_E);
    o.key[K_CHI_U] = hkey(s, id, P_CHI_U);
    o.key[K_CHI_D] = hkey(s, id, P_CHI_D);
    auto cp = [&](u128 *dst[MAXP], ct_u128 *const src[CT_MAX_PARTIES]) {
        for (int q = 0; q < c->np; q++) dst[q] = reinterpret_cast<u128 *>(src[q]);
    };
    cp(o.X, b.X); cp(o.tX, b.tX); cp(o.A, b.A); cp(o.tA, b.tA);
    cp(o.Y, b.Y); cp(o.tY, b.tY); cp(o.B, b.B); cp(o.tB, b.tB);
    cp(o.C, b.C); cp(o.tC, b.tC); cp(o.R, b.R); cp(o.tR, b.tR);
    cp(o.Z, b.Z); cp(o.tZ, b.tZ);
    cp(o.Rf, b.Rf); cp(o.tRf, b.tRf); cp(o.Zf, b.Zf); cp(o.tZf, b.tZf);
    o.f = d.f;
    o.in_bits = d.in_bits;
    o.cm = CT_COMPRESS_ALONG_M(d.M, d.N, d.compress) ? 1 : 0;
    if (d.conv_c > 0) {
        o.cv.on = 1;
        o.cv.c = d.conv_c; o.cv.h = d.conv_h; o.cv.w = d.conv_w;
        o.cv.k = d.conv_k; o.cv.s = d.conv_stride; o.cv.p = d.conv_pad;
        o.cv.wo = (d.conv_w + 2 * d.conv_pad - d.conv_k) / d.conv_stride + 1;
    }
    o.nr = CT_RIGHT_LEN(d);
    o.E = reinterpret_cast<u128 *>(b.E);
    o.U = reinterpret_cast<u128 *>(b.U);
    o.D = reinterpret_cast<u128 *>(b.D);
    o.cvec = reinterpret_cast<u128 *>(b.cvec);
    o.work = reinterpret_cast<u128 *>(b.work);
    o.acc = acc + (size_t)l * ACC_PER_LAYER;
}

struct Sizes {
    int64_t mk = 0, kn = 0, mn = 0, m = 0, k = 0, cvec = 0, kn_items = 0, mn_items = 0, row_items = 0,
            skinny_mn = 0, col_tag = 0, nr = 0, conv_items = 0;
    bool skinny = false, cm = false, conv_n = false;
};

Sizes max_sizes(const ct_layer_desc *L, int n) {
    Sizes s;
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        s.mk = std::max(s.mk, d.M * d.K);
        s.kn = std::max(s.kn, d.K * d.N);
        s.mn = std::max(s.mn, d.M * d.N);
        s.m = std::max(s.m, d.M);
        s.k = std::max(s.k, d.K);
        s.cvec = std::max(s.cvec, (int64_t)CT_CVEC_LEN_FOR(d.M, d.K, d.N, d.compress));
        // a convolution's U is opened elementwise on its input (about 4 elements per lane)
        s.kn_items = std::max(s.kn_items, d.conv_c > 0 ? (int64_t)CT_RIGHT_LEN(d) / 256 + 1 : sweep_items(d.K, d.N));
        s.mn_items = std::max(s.mn_items, sweep_items(d.M, d.N));
        s.row_items = std::max(s.row_items, row_items(d.M, d.K));
        s.nr = std::max(s.nr, (int64_t)CT_RIGHT_LEN(d));
        if (d.conv_c > 0 && !CT_COMPRESS_ALONG_M(d.M, d.N, d.compress)) {
            // compression of the implicit im2col matrices along N
            s.conv_n = true;
            s.conv_items = std::max(s.conv_items, conv_compress_items(d.conv_c, d.N));
        }
        if (CT_COMPRESS_ALONG_M(d.M, d.N, d.compress)) {
            // column-strip row pass, column sweeps of the M x N pass and of the compact products
            s.cm = true;
            s.row_items = std::max(s.row_items, cm_items(d.M, d.K, d.N));
            s.mn_items = std::max(s.mn_items, col_sweep_items(d.M, d.N));
            s.col_tag = std::max(s.col_tag, col_sweep_items(d.K, d.N));
        }
        if (d.N <= SKINNY_MAX_N) {
            s.skinny = true;
            s.skinny_mn = std::max(s.skinny_mn, d.M * d.N);
        }
    }
    return s;
}

// Waits for the lane's previous upload, then stages the layer records.
// out_index: position of each layer's check record in the caller's result
// array (null: the layer's own position).
ct_status stage_layers(ct_ctx *c, Lane &ln, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                       const int *out_index = nullptr) {
    HIPCHK(c, hipEventSynchronize(ln.upload_done));
    for (int l = 0; l < n; l++) {
        fill_layer(c, ln.acc_dev, L[l], B[l], l, ln.layers_host[l]);
        ln.layers_host[l].out_index = out_index ? out_index[l] : l;
    }
    return CT_OK;
}

ct_status upload(ct_ctx *c, Lane &ln, int n, int nprobs, int njobs = 0, int nskinny = 0) {
    HIPCHK(c, hipMemcpyAsync(ln.layers_dev, ln.layers_host, sizeof(LayerDev) * n, hipMemcpyHostToDevice, ln.stream));
    if (nprobs > 0)
        HIPCHK(c, hipMemcpyAsync(ln.gemm_dev, ln.gemm_host, sizeof(GemmProb) * nprobs, hipMemcpyHostToDevice,
                                 ln.stream));
    if (njobs > 0)
        HIPCHK(c, hipMemcpyAsync(ln.pack_dev, ln.pack_host, sizeof(PackJob) * njobs, hipMemcpyHostToDevice,
                                 ln.stream));
    if (nskinny > 0)
        HIPCHK(c, hipMemcpyAsync(ln.skinny_dev, ln.skinny_host, sizeof(SkinnyProb) * nskinny,
                                 hipMemcpyHostToDevice, ln.stream));
    HIPCHK(c, hipEventRecord(ln.upload_done, ln.stream));
    return CT_OK;
}

// Element e of a buffer of the context's ring (eb bytes per element): the
// tables hold u128 pointers whatever the element width, so offsets are
// applied in bytes.
inline u128 *elem_at(u128 *base, int64_t e, int eb) {
    return reinterpret_cast<u128 *>(reinterpret_cast<char *>(base) + e * (int64_t)eb);
}

// Host-side bound check of a layer's workspace use: every packed operand
// (tiles * TILE_ELEMS elements from dst) must end inside the caller's
// CT_WORK_LEN(M, K, N) elements.
bool job_in_work(const PackJob &j, const u128 *work, const ct_layer_desc &d, int eb, int np = 2) {
    const char *b = reinterpret_cast<const char *>(work);
    const char *e = reinterpret_cast<const char *>(j.dst) + (int64_t)j.tiles * TILE_ELEMS * eb;
    return reinterpret_cast<const char *>(j.dst) >= b && e <= b + (int64_t)CT_WORK_LEN_NP(d.M, d.K, d.N, np) * eb;
}

// Workspace of a matrix-core layer with n parties: the folded operands
// A_0 + E and [tA]_p + [Delta]_p E (M K each), then 2n + 1 packed left
// operands (E, A_0 + E, [A]_1 .. [A]_{n-1}, [tA]_p + [Delta]_p E) and 2n + 1
// packed right ones ([B]_p, U, [tB]_p).
struct NpWork {
    int64_t mk, pl, pr;
    int np;
    int64_t fold_tA(int p) const { return (1 + p) * mk; }
    int64_t left(int i) const { return (1 + np) * mk + i * pl; }
    int64_t right(int j) const { return (1 + np) * mk + (2 * np + 1) * pl + j * pr; }
};
NpWork np_work(int64_t M, int64_t K, int64_t N, int np) {
    NpWork w;
    w.mk = M * K; w.pl = packed_elems(M, K); w.pr = packed_elems(N, K); w.np = np;
    return w;
}

GemmProb make_prob(const u128 *Lp1, const u128 *Lp2, const u128 *Rp1, const u128 *Rp2, const u128 *base, u128 *out,
                   const ct_layer_desc &d) {
    GemmProb p;
    std::memset(&p, 0, sizeof(p));
    p.Lp1 = Lp1; p.Lp2 = Lp2; p.Rp1 = Rp1; p.Rp2 = Rp2; p.base = base; p.out = out;
    p.M = (int32_t)d.M; p.N = (int32_t)d.N; p.K = (int32_t)d.K;
    p.gsize = 1;
    return p;
}

PackJob make_job(const u128 *src, u128 *dst, int64_t rows, int64_t cols, int side, const ConvGeom *cv = nullptr) {
    PackJob j;
    std::memset(&j, 0, sizeof(j));
    j.src = src; j.dst = dst; j.rows = (int32_t)rows; j.cols = (int32_t)cols; j.side = side;
    if (cv && side == 1) j.cv = *cv;
    const int64_t major = side == 0 ? rows : cols, K = side == 0 ? cols : rows;
    j.majt = (int32_t)((major + 63) / 64);
    j.kt = (int32_t)((K + 31) / 32);
    j.tiles = j.majt * j.kt;
    return j;
}

// Assigns tile ranges to packing jobs; returns the total tile count.
int plan_jobs(PackJob *jobs, int njobs) {
    int t = 0;
    for (int i = 0; i < njobs; i++) {
        jobs[i].tile_begin = t;
        t += jobs[i].tiles;
    }
    return t;
}

// Orders MFMA problems first, then skinny ones; assigns tiles and K splits.
// Returns the number of MFMA problems; *total_tiles receives their tile count.
constexpr int MAX_STEPS_PER_SPLIT = 255;  // keeps every int32 diagonal exact

// Shape class of a call: the protocol and, per matrix-core layer, the
// rounded-up binary logarithms of M, K and N (FNV-1a hash).
uint64_t shape_class(int mode, const ct_layer_desc *L, int n) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    auto lg = [](int64_t v) { int r = 0; while ((1LL << r) < v) r++; return (uint64_t)r; };
    mix((uint64_t)mode);
    for (int l = 0; l < n; l++)
        if (L[l].N > SKINNY_MAX_N) mix((lg(L[l].M) << 16) | (lg(L[l].K) << 8) | lg(L[l].N));
    return h;
}

GemmTuning tuning_for(const ct_ctx *c, uint64_t key) {
    if (c->forcing) return c->forced;
    auto it = c->tuned.find(key);
    return it == c->tuned.end() ? c->fallback : it->second;
}

// Plans the products: probs holds consecutive groups (the products of one
// layer); gsize of each problem must be set.  Fills tiles, K splits and the
// group tile ranges.
// Output tiles per wavefront (stacked in M) a launch takes: tuning tile
// shapes 128 x 64 exist for Z_{2^64} only (8 diagonal accumulators per tile
// leave room for two); CT_TILE_AUTO takes them when the launch still has two
// such workgroup tiles per compute unit before any K split.
int gemm_mt(const std::vector<GemmProb> &probs, int num_cus, const GemmTuning &tu, int eb) {
    if (eb != 8) return 1;
    if (tu.tile == CT_TILE_LDS_128x64 || tu.tile == CT_TILE_REGS_128x64) return 2;
    if (tu.tile != CT_TILE_AUTO) return 1;
    int64_t tiles128 = 0;
    for (const auto &p : probs) tiles128 += (int64_t)((p.M + 127) / 128) * ((p.N + 63) / 64);
    return tiles128 >= 2LL * num_cus ? 2 : 1;
}
int gemm_kernel(const GemmTuning &tu) {
    return tu.tile == CT_TILE_LDS_64x64 || tu.tile == CT_TILE_LDS_128x64 ? GEMM_LDS : GEMM_REGS;
}

// CT_TILE_REGS_FIT: the workgroup tile of a product with the fewest padded
// outputs, 64 x 64 on ties (its four wavefronts share two left and two right
// fragments; the narrow shapes read five).
int fit_wshape(int M, int N) {
    auto padded = [&](int wm, int wn) { return (int64_t)((M + wm - 1) / wm * wm) * ((N + wn - 1) / wn * wn); };
    const int64_t sq = padded(64, 64), wide = padded(32, 128), tall = padded(128, 32);
    if (wide < sq && wide <= tall) return WS_32x128;
    if (tall < sq) return WS_128x32;
    return WS_64x64;
}

int plan_gemms(std::vector<GemmProb> &probs, int num_cus, const GemmTuning &tu, int *total_tiles, bool *any_accum,
               int eb) {
    const int mt = gemm_mt(probs, num_cus, tu, eb);
    int64_t total_steps = 0;
    for (auto &p : probs) {
        p.mt = mt;
        p.wshape = tu.tile == CT_TILE_REGS_FIT ? fit_wshape(p.M, p.N) : WS_64x64;
        const int wgm = p.wshape == WS_32x128 ? 32 : p.wshape == WS_128x32 ? 128 : 64 * mt;
        const int wgn = p.wshape == WS_32x128 ? 128 : p.wshape == WS_128x32 ? 32 : 64;
        p.tiles_m = (p.M + wgm - 1) / wgm;
        p.tiles_n = (p.N + wgn - 1) / wgn;
        p.kt = (p.K + 31) / 32;
        p.nsteps = p.kt * (p.Lp2 ? 2 : 1);
        p.group_m = std::max(1, std::min(tu.group_m, p.tiles_m));
        total_steps += (int64_t)p.tiles_m * p.tiles_n * p.nsteps;
    }
    // K slices per tile: by default enough tiles for two rounds over the
    // compute units, equal-length tiles across problems; at least 8 slices
    // per tile (split partials cost atomics), at most MAX_STEPS_PER_SPLIT
    // (exactness of the int32 diagonals).
    int64_t target = tu.split_target > 0 ? tu.split_target : (total_steps + 2LL * num_cus - 1) / (2LL * num_cus);
    if (target < 8) target = 8;
    if (target > MAX_STEPS_PER_SPLIT) target = MAX_STEPS_PER_SPLIT;
    int tile = 0;
    *any_accum = false;
    for (size_t i = 0; i < probs.size();) {
        const int gs = probs[i].gsize;
        GemmProb &p0 = probs[i];
        const int64_t splits = std::max<int64_t>(1, (p0.nsteps + target - 1) / target);
        const int sps = (int)((p0.nsteps + splits - 1) / splits);
        const int nspl = (p0.nsteps + sps - 1) / sps;
        const int gtiles = p0.tiles_m * p0.tiles_n * nspl * gs;
        for (int j = 0; j < gs; j++) {
            GemmProb &p = probs[i + j];
            p.steps_per_split = sps;
            p.splits = nspl;
            p.accumulate = nspl > 1 ? 1 : 0;
            p.tile_begin = tile;
            p.tiles = gtiles;
            p.gfirst = (int)i;
        }
        if (nspl > 1) *any_accum = true;
        tile += gtiles;
        i += gs;
    }
    *total_tiles = tile;
    return (int)probs.size();
}

ct_status run_gemms(ct_ctx *c, Lane &ln, int nprobs, int total_tiles, const GemmTuning &tu) {
    if (nprobs > 0)
        LAUNCH(c, ln, ST_RING_GEMM, launch_gemm(c->eb, ln.gemm_dev, nprobs, total_tiles, tu.xcd_remap,
                                                ln.gemm_host[0].mt, gemm_kernel(tu), ln.stream));
    return CT_OK;
}

}  // namespace

namespace ct {

ct_status fail(ct_ctx *c, ct_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

hipError_t lane_init(Lane &ln, hipStream_t stream, int max_layers) {
    ln.stream = stream;
    ln.max_layers = max_layers;
    // up to two products per party and 4 n + 2 packed operands per layer
    ln.max_probs = 2 * CT_MAX_PARTIES * max_layers;
    ln.max_jobs = (4 * CT_MAX_PARTIES + 2) * max_layers;
    hipError_t e;
#define LANE_TRY(expr) \
    if ((e = (expr)) != hipSuccess) return e
    LANE_TRY(hipMalloc(&ln.layers_dev, sizeof(LayerDev) * ln.max_layers));
    LANE_TRY(hipMalloc(&ln.gemm_dev, sizeof(GemmProb) * ln.max_probs));
    LANE_TRY(hipMalloc(&ln.pack_dev, sizeof(PackJob) * ln.max_jobs));
    LANE_TRY(hipMalloc(&ln.skinny_dev, sizeof(SkinnyProb) * ln.max_layers));
    LANE_TRY(hipMalloc(&ln.acc_dev, sizeof(u128) * ACC_PER_LAYER * ln.max_layers));
    LANE_TRY(hipMalloc(&ln.res_dev, sizeof(ct_check_result) * ln.max_layers));
    LANE_TRY(hipMalloc(&ln.sync_dev, 64));
    LANE_TRY(hipHostMalloc(&ln.layers_host, sizeof(LayerDev) * ln.max_layers, hipHostMallocDefault));
    LANE_TRY(hipHostMalloc(&ln.gemm_host, sizeof(GemmProb) * ln.max_probs, hipHostMallocDefault));
    LANE_TRY(hipHostMalloc(&ln.pack_host, sizeof(PackJob) * ln.max_jobs, hipHostMallocDefault));
    LANE_TRY(hipHostMalloc(&ln.skinny_host, sizeof(SkinnyProb) * ln.max_layers, hipHostMallocDefault));
    LANE_TRY(hipHostMalloc(&ln.res_host, sizeof(ct_check_result) * ln.max_layers, hipHostMallocDefault));
    LANE_TRY(hipEventCreateWithFlags(&ln.upload_done, hipEventDisableTiming));
    LANE_TRY(hipEventRecord(ln.upload_done, ln.stream));
#undef LANE_TRY
    return hipSuccess;
}

void lane_free(Lane &ln) {
    if (ln.upload_done) (void)hipEventDestroy(ln.upload_done);
    if (ln.sync_dev) (void)hipFree(ln.sync_dev);
    if (ln.layers_dev) (void)hipFree(ln.layers_dev);
    if (ln.gemm_dev) (void)hipFree(ln.gemm_dev);
    if (ln.pack_dev) (void)hipFree(ln.pack_dev);
    if (ln.skinny_dev) (void)hipFree(ln.skinny_dev);
    if (ln.acc_dev) (void)hipFree(ln.acc_dev);
    if (ln.res_dev) (void)hipFree(ln.res_dev);
    if (ln.layers_host) (void)hipHostFree(ln.layers_host);
    if (ln.gemm_host) (void)hipHostFree(ln.gemm_host);
    if (ln.pack_host) (void)hipHostFree(ln.pack_host);
    if (ln.skinny_host) (void)hipHostFree(ln.skinny_host);
    if (ln.res_host) (void)hipHostFree(ln.res_host);
    ln = Lane();
}

}  // namespace ct

extern "C" {

ct_status ct_create(ct_ctx **out, const ct_params *p) {
    if (!out || !p) return CT_EINVAL;
    *out = nullptr;
    if (!((p->k_bits == 64 && p->s_bits == 64) || (p->k_bits == 32 && p->s_bits == 32))) return CT_EINVAL;
    ct_ctx *c = new ct_ctx();
    c->device = p->device;
    c->eb = p->k_bits == 32 ? 8 : 16;
    if (p->parties != 0 && (p->parties < 2 || p->parties > CT_MAX_PARTIES)) {
        delete c;
        return CT_EINVAL;
    }
    c->np = p->parties == 0 ? 2 : p->parties;
    // F_MAC Initialize: [Delta]_p uniform in Z_{2^s} (the key draw mod 2^s)
    for (int q = 0; q < c->np; q++) {
        const uint64_t x = hdraw(hkey(p->key_seed, GLOBAL_LAYER, P_KEY + q), 0);
        c->delta[q] = p->s_bits == 32 ? (x & 0xFFFFFFFFull) : x;
    }
    hipError_t e;
    if ((e = hipSetDevice(c->device)) == hipSuccess) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
            c->num_cus = cus;
        const int ml = p->max_layers > 0 ? p->max_layers : 256;
        e = lane_init(c->main, reinterpret_cast<hipStream_t>(p->hip_stream), ml);
        hipStream_t side = nullptr;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
        if (e == hipSuccess) e = lane_init(c->side, side, ml);
        else c->side.stream = side;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
        if (e == hipSuccess) e = scratch_address(c->device, &c->static_work);
        if (e == hipSuccess) c->static_bufs.resize(ml);
    }
    if (e != hipSuccess) {
        std::fprintf(stderr, "ct_create: %s\n", hipGetErrorString(e));
        ct_destroy(c);
        return CT_EDEVICE;
    }
    c->main.timed = true;
    *out = c;
    return CT_OK;
}

ct_status ct_destroy(ct_ctx *c) {
    if (!c) return CT_EINVAL;
    if (c->main.layers_dev) (void)hipStreamSynchronize(c->main.stream);
    if (c->side.stream) (void)hipStreamSynchronize(c->side.stream);
    for (auto e : c->ev_start) (void)hipEventDestroy(e);
    for (auto e : c->ev_end) (void)hipEventDestroy(e);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->join) (void)hipEventDestroy(c->join);
    lane_free(c->main);
    hipStream_t side = c->side.stream;
    lane_free(c->side);
    if (side) (void)hipStreamDestroy(side);
    delete c;
    return CT_OK;
}

ct_status ct_key_shares(const ct_ctx *c, uint64_t out[CT_MAX_PARTIES]) {
    if (!c || !out) return CT_EINVAL;
    for (int q = 0; q < c->np; q++) out[q] = c->delta[q];
    return CT_OK;
}

const char *ct_last_error(const ct_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

ct_status ct::run_deal(ct_ctx *c, Lane &ln, const ct_layer_desc *L, const ct_layer_bufs *B, int n, int with_inputs) {
    ct_status s = validate(c, ln.max_layers, L, B, n, NEED_TRIPLE | NEED_WORK | (with_inputs ? NEED_INPUTS : 0));
    if (s != CT_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = stage_layers(c, ln, L, B, n)) != CT_OK) return s;
    // C~ = A~ B~ with the lifts left in party 1's buffers: packed matrix-core
    // product for wide layers (operand tiles in the workspace), VALU rows for
    // layers with N <= SKINNY_MAX_N.
    std::vector<GemmProb> probs;
    int njobs = 0, nskinny = 0;
    const int last = c->np - 1;  // the lifts go to the last party's buffers
    for (int l = 0; l < n; l++) {
        const LayerDev &o = ln.layers_host[l];
        const ct_layer_desc &d = L[l];
        if (d.N <= SKINNY_MAX_N) {
            SkinnyProb sp;
            std::memset(&sp, 0, sizeof(sp));
            sp.L = o.A[last]; sp.R = o.B[last]; sp.out = o.C[last];
            sp.M = (int32_t)d.M; sp.N = (int32_t)d.N; sp.K = (int32_t)d.K;
            ln.skinny_host[nskinny++] = sp;
            continue;
        }
        const WorkOff w = work_off(d.M, d.K, d.N);
        u128 *Ep = elem_at(o.work, w.Ep, c->eb), *B0p = elem_at(o.work, w.B0p, c->eb);
        ln.pack_host[njobs++] = make_job(o.A[last], Ep, d.M, d.K, 0);
        ln.pack_host[njobs++] = make_job(o.B[last], B0p, d.K, d.N, 1, &o.cv);
        if (!job_in_work(ln.pack_host[njobs - 2], o.work, d, c->eb, c->np) ||
            !job_in_work(ln.pack_host[njobs - 1], o.work, d, c->eb, c->np))
            return fail(c, CT_EINVAL, "internal error: workspace layout exceeds CT_WORK_LEN");
        probs.push_back(make_prob(Ep, nullptr, B0p, nullptr, nullptr, o.C[last], d));
    }
    const int pack_tiles = plan_jobs(ln.pack_host, njobs);
    int total_tiles = 0;
    bool any_accum = false;
    const GemmTuning tu = c->fallback;
    const int nm = plan_gemms(probs, c->num_cus, tu, &total_tiles, &any_accum, c->eb);
    std::copy(probs.begin(), probs.end(), ln.gemm_host);
    if ((s = upload(c, ln, n, nm, njobs, nskinny)) != CT_OK) return s;
    const Sizes sz = max_sizes(L, n);
    if (c->np > 2) LAUNCH(c, ln, ST_DEAL_LIFT, launch_np_lift(c->eb, ln.layers_dev, n, std::max(sz.mk, sz.nr), ln.stream));
    else LAUNCH(c, ln, ST_DEAL_LIFT, launch_deal_lift(c->eb, ln.layers_dev, n, std::max(sz.mk, sz.nr), ln.stream));
    LAUNCH(c, ln, ST_PACK, launch_pack(c->eb, ln.pack_dev, njobs, pack_tiles, ln.stream));
    for (int i = 0; i < nm; i++)
        if (probs[i].accumulate)
            LAUNCH(c, ln, ST_FILL_ZERO, launch_fill_zero(c->eb, probs[i].out, (int64_t)probs[i].M * probs[i].N, ln.stream));
    if ((s = run_gemms(c, ln, nm, total_tiles, tu)) != CT_OK) return s;
    if (nskinny > 0) {
        int max_rows = 0;
        for (int i = 0; i < nskinny; i++) max_rows = std::max(max_rows, ln.skinny_host[i].M);
        LAUNCH(c, ln, ST_DEAL_SKINNY, launch_skinny(c->eb, ln.skinny_dev, nskinny, max_rows, ln.stream));
    }
    const int mask = (with_inputs ? ((1 << OBJ_X) | (1 << OBJ_Y)) : 0) | (1 << OBJ_A) | (1 << OBJ_B) |
                     (1 << OBJ_C) | (1 << OBJ_R) | (1 << OBJ_RF);
    if (c->np > 2)
        LAUNCH(c, ln, ST_DEAL_AUTH, launch_np_auth(c->eb, ln.layers_dev, n, mask, std::max({sz.mk, sz.nr, sz.mn}), ln.stream));
    else
        LAUNCH(c, ln, ST_DEAL_AUTH, launch_deal_auth(c->eb, ln.layers_dev, n, mask, std::max({sz.mk, sz.nr, sz.mn}), ln.stream));
    return CT_OK;
}


extern "C" {

ct_status ct_gen_triple_tags(ct_ctx *c, const ct_layer_desc *L, const ct_layer_bufs *B, int n, int with_inputs) {
    if (!c) return CT_EINVAL;
    return run_deal(c, c->main, L, B, n, with_inputs);
}

}  // extern "C"

namespace ct {

// ---- n parties (np > 2): the plain per-step passes of ct_parties.hip and one
// matrix-core product per party (two in SPDZ2k mode):
//   [Z]_p = [C]_p + E [B]_p + L_p U,  L_0 = A_0 + E, L_p = [A]_p;
//   [tZ]_p = [tC]_p + E [tB]_p + ([tA]_p + [Delta]_p E) U.
ct_status prepare_online_np(ct_ctx *c, Lane &ln, ct_mode mode, const ct_layer_desc *L, int n,
                            ct_check_result *out_dev, OnlineLaunch &P) {
    const bool compact = mode == CT_MODE_COMPACT, check = out_dev != nullptr;
    const int np = c->np;
    std::vector<GemmProb> probs;
    int njobs = 0;
    PackJob *J = ln.pack_host;
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        if (d.N <= SKINNY_MAX_N) continue;
        const LayerDev &o = ln.layers_host[l];
        const NpWork w = np_work(d.M, d.K, d.N, np);
        if (njobs + 4 * np + 2 > ln.max_jobs || (int)probs.size() + 2 * np > ln.max_probs)
            return fail(c, CT_EINVAL, "internal error: layer tables too small");
        auto wp = [&](int64_t e) { return elem_at(o.work, e, c->eb); };
        const int first_job = njobs;
        J[njobs++] = make_job(o.E, wp(w.left(0)), d.M, d.K, 0);
        J[njobs++] = make_job(wp(0), wp(w.left(1)), d.M, d.K, 0);  // A_0 + E
        for (int p = 1; p < np; p++) J[njobs++] = make_job(o.A[p], wp(w.left(1 + p)), d.M, d.K, 0);
        for (int p = 0; p < np; p++) J[njobs++] = make_job(o.B[p], wp(w.right(p)), d.K, d.N, 1);
        J[njobs++] = make_job(o.U, wp(w.right(np)), d.K, d.N, 1);
        const size_t first = probs.size();
        for (int p = 0; p < np; p++)
            probs.push_back(make_prob(wp(w.left(0)), wp(w.left(1 + p)), wp(w.right(p)), wp(w.right(np)), o.C[p], o.Z[p], d));
        if (!compact) {
            for (int p = 0; p < np; p++) {
                J[njobs++] = make_job(wp(w.fold_tA(p)), wp(w.left(np + 1 + p)), d.M, d.K, 0);
                J[njobs++] = make_job(o.tB[p], wp(w.right(np + 1 + p)), d.K, d.N, 1);
                probs.push_back(make_prob(wp(w.left(0)), wp(w.left(np + 1 + p)), wp(w.right(np + 1 + p)),
                                          wp(w.right(np)), o.tC[p], o.tZ[p], d));
            }
        }
        for (size_t j = first; j < probs.size(); j++) probs[j].gsize = (int32_t)(probs.size() - first);
        for (int j = first_job; j < njobs; j++)
            if (!job_in_work(J[j], o.work, d, c->eb, np))
                return fail(c, CT_EINVAL, "internal error: workspace layout exceeds CT_WORK_LEN_NP");
    }
    P = OnlineLaunch();
    P.n = n;
    P.mode = mode;
    P.compact = compact;
    P.check = check;
    P.out_dev = out_dev;
    P.njobs = njobs;
    P.pack_tiles = plan_jobs(ln.pack_host, njobs);
    P.tu = tuning_for(c, shape_class(mode, L, n));
    P.nm = plan_gemms(probs, c->num_cus, P.tu, &P.total_tiles, &P.any_accum, c->eb);
    std::copy(probs.begin(), probs.end(), ln.gemm_host);
    ct_status s = upload(c, ln, n, P.nm, njobs);
    if (s != CT_OK) return s;
    P.flags = (check ? F_CHECK : 0) | (compact ? F_COMPACT : F_SPDZ);
    bool fused_skinny = false;
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        P.max_open = std::max({P.max_open, d.M * d.K, d.K * d.N});
        P.max_mn = std::max(P.max_mn, d.M * d.N);
        P.max_compress_items = std::max(P.max_compress_items, sweep_items(d.M, d.N));
        P.max_cvec_np = std::max(P.max_cvec_np, (int64_t)CT_CVEC_LEN_NP(d.M, d.K, np));
        if (np_fused_row(d.N)) {
            // the fused row pass (variants 0, 1, 2)
            P.variants |= 1 << row_variant(d.N);
            P.max_row_items = std::max(P.max_row_items, row_items(d.M, d.K));
            if (d.N <= SKINNY_MAX_N) {
                fused_skinny = true;
                P.max_zero = std::max(P.max_zero, d.M * d.N);
            }
        } else {
            P.any_unfused = true;
            P.max_gemv_items = std::max(P.max_gemv_items, sweep_items(d.M, d.K));
            P.max_skinny_items = std::max(P.max_skinny_items, d.M * np);
        }
    }
    P.max_zero = std::max(P.max_zero, compact ? P.max_cvec_np : 0);
    P.zero_what = (compact ? 1 : 0) | (check ? 2 : 0) | (fused_skinny ? 4 : 0) | (fused_skinny && !compact ? 8 : 0);
    return CT_OK;
}

ct_status enqueue_online_np(ct_ctx *c, Lane &ln, const OnlineLaunch &P) {
    const int n = P.n;
    if (P.zero_what)
        LAUNCH(c, ln, ST_ZERO_ACC, launch_np_zero(c->eb, ln.layers_dev, n, P.zero_what, P.max_zero, ln.stream));
    // U and its compression (formed by the same pass) first: the fused row
    // pass reads U^c, [tB^c]_p and, for N <= 2, U
    LAUNCH(c, ln, ST_OPEN_U, launch_np_open(c->eb, ln.layers_dev, n, 2, P.flags, P.max_open, ln.stream));
    if (P.variants)
        LAUNCH(c, ln, ST_ROW_PASS,
               launch_np_row_pass(c->eb, c->np, ln.layers_dev, n, P.flags, P.max_row_items, P.variants, ln.stream));
    if (P.any_unfused) LAUNCH(c, ln, ST_NP_OPEN, launch_np_open(c->eb, ln.layers_dev, n, 1, P.flags, P.max_open, ln.stream));
    if (P.njobs > 0) LAUNCH(c, ln, ST_PACK, launch_pack(c->eb, ln.pack_dev, P.njobs, P.pack_tiles, ln.stream));
    if (P.any_accum) LAUNCH(c, ln, ST_COPY_BASE, launch_prob_base(c->eb, ln.gemm_dev, P.nm, P.max_mn, ln.stream));
    ct_status s = run_gemms(c, ln, P.nm, P.total_tiles, P.tu);
    if (s != CT_OK) return s;
    if (P.any_unfused)
        LAUNCH(c, ln, ST_NP_SKINNY, launch_np_skinny(c->eb, ln.layers_dev, n, P.flags, P.max_skinny_items, ln.stream));
    LAUNCH(c, ln, ST_POST, launch_np_post(c->eb, ln.layers_dev, n, P.flags, P.max_mn, ln.stream));
    if (P.compact) {
        LAUNCH(c, ln, ST_NP_COMPRESS, launch_np_compress(c->eb, ln.layers_dev, n, P.max_compress_items, ln.stream));
        if (P.any_unfused)
            LAUNCH(c, ln, ST_NP_GEMV, launch_np_gemv(c->eb, ln.layers_dev, n, P.max_gemv_items, ln.stream));
        LAUNCH(c, ln, ST_COMPACT_FINAL, launch_np_compact_final(c->eb, ln.layers_dev, n, P.flags, ln.stream));
    }
    if (P.check) LAUNCH(c, ln, ST_FINALIZE, launch_np_finalize(c->eb, ln.layers_dev, n, P.out_dev, ln.stream));
    return CT_OK;
}

// The online phase, optionally with the verification fused into its passes
// (out_dev != nullptr): validation, tables and their upload.
ct_status prepare_online(ct_ctx *c, Lane &ln, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                         ct_check_result *out_dev, OnlineLaunch &P, const int *out_index) {
    if (!c) return CT_EINVAL;
    if (mode != CT_MODE_SPDZ2K && mode != CT_MODE_COMPACT) return fail(c, CT_EINVAL, "unknown mode");
    const bool compact = mode == CT_MODE_COMPACT;
    const bool check = out_dev != nullptr;
    ct_status s = validate(c, ln.max_layers, L, B, n,
                           NEED_INPUTS | NEED_TRIPLE | NEED_OUT | NEED_WORK | (compact ? NEED_CVEC : 0));
    if (s != CT_OK) return s;
    if (check && !aligned16(out_dev)) return fail(c, CT_EINVAL, "out_dev is null or misaligned");
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = stage_layers(c, ln, L, B, n, out_index)) != CT_OK) return s;
    if (c->np > 2) return prepare_online_np(c, ln, mode, L, n, out_dev, P);

    // Matrix-core products (layers with N > SKINNY_MAX_N), both parties,
    // Eq. (2) with E U folded into party 0's left operand by the row pass:
    //   [Z]_0 = [C]_0 + E [B]_0 + (A_0 + E) U,   [Z]_1 = [C]_1 + E [B]_1 + [A]_1 U;
    // SPDZ2k tags of Eq. (3):  [tZ]_p = [tC]_p + E [tB]_p + ([tA]_p + [Delta]_p E) U.
    // Every operand is converted once into digit tiles in the workspace.
    std::vector<GemmProb> probs;
    probs.reserve(4 * n);
    int njobs = 0;
    int64_t open_tiles = 0;
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        if (d.N <= SKINNY_MAX_N) continue;
        const LayerDev &o = ln.layers_host[l];
        const WorkOff w = work_off(d.M, d.K, d.N);
        u128 *W = o.work;
        auto wp = [&](int64_t e) { return elem_at(W, e, c->eb); };
        const int first_job = njobs;
        PackJob *J = ln.pack_host;
        J[njobs++] = make_job(o.E, wp(w.Ep), d.M, d.K, 0);
        J[njobs++] = make_job(wp(w.AE0), wp(w.AE0p), d.M, d.K, 0);
        J[njobs++] = make_job(o.A[1], wp(w.A1p), d.M, d.K, 0);
        if (!o.cv.on) {
            // k_open_pack opens U and writes the right operands' digit tiles
            const PackJob rj[3] = {make_job(o.B[0], wp(w.B0p), d.K, d.N, 1), make_job(o.B[1], wp(w.B1p), d.K, d.N, 1),
                                   make_job(o.U, wp(w.Up), d.K, d.N, 1)};
            for (const PackJob &j : rj)
                if (!job_in_work(j, W, d, c->eb))
                    return fail(c, CT_EINVAL, "internal error: workspace layout exceeds CT_WORK_LEN");
            LayerDev &lh = ln.layers_host[l];
            lh.fo = 1;
            lh.rp[0] = wp(w.B0p);
            lh.rp[1] = wp(w.B1p);
            lh.rp[2] = wp(w.Up);
            open_tiles = std::max<int64_t>(open_tiles, rj[0].tiles);
        } else {
            J[njobs++] = make_job(o.B[0], wp(w.B0p), d.K, d.N, 1, &o.cv);
            J[njobs++] = make_job(o.B[1], wp(w.B1p), d.K, d.N, 1, &o.cv);
            J[njobs++] = make_job(o.U, wp(w.Up), d.K, d.N, 1, &o.cv);
        }
        const size_t first = probs.size();
        probs.push_back(make_prob(wp(w.Ep), wp(w.AE0p), wp(w.B0p), wp(w.Up), o.C[0], o.Z[0], d));
        probs.push_back(make_prob(wp(w.Ep), wp(w.A1p), wp(w.B1p), wp(w.Up), o.C[1], o.Z[1], d));
        if (!compact) {
            J[njobs++] = make_job(wp(w.tAE0), wp(w.tAE0p), d.M, d.K, 0);
            J[njobs++] = make_job(wp(w.tAE1), wp(w.tAE1p), d.M, d.K, 0);
            J[njobs++] = make_job(o.tB[0], wp(w.tB0p), d.K, d.N, 1, &o.cv);
            J[njobs++] = make_job(o.tB[1], wp(w.tB1p), d.K, d.N, 1, &o.cv);
            probs.push_back(make_prob(wp(w.Ep), wp(w.tAE0p), wp(w.tB0p), wp(w.Up), o.tC[0], o.tZ[0], d));
            probs.push_back(make_prob(wp(w.Ep), wp(w.tAE1p), wp(w.tB1p), wp(w.Up), o.tC[1], o.tZ[1], d));
        }
        for (size_t j = first; j < probs.size(); j++) probs[j].gsize = (int32_t)(probs.size() - first);
        for (int j = first_job; j < njobs; j++)  // every packed operand lies inside the workspace
            if (!job_in_work(J[j], W, d, c->eb))
                return fail(c, CT_EINVAL, "internal error: workspace layout exceeds CT_WORK_LEN");
    }
    P = OnlineLaunch();
    P.n = n;
    P.mode = mode;
    P.compact = compact;
    P.check = check;
    P.out_dev = out_dev;
    P.njobs = njobs;
    P.open_tiles = (int)open_tiles;
    for (int l = 0; l < n; l++) P.any_open_u |= !ln.layers_host[l].fo;
    P.pack_tiles = plan_jobs(ln.pack_host, njobs);
    P.tu = tuning_for(c, shape_class(mode, L, n));
    P.nm = plan_gemms(probs, c->num_cus, P.tu, &P.total_tiles, &P.any_accum, c->eb);
    std::copy(probs.begin(), probs.end(), ln.gemm_host);
    if ((s = upload(c, ln, n, P.nm, njobs)) != CT_OK) return s;

    const Sizes sz = max_sizes(L, n);
    P.max_zero = std::max(compact ? sz.cvec : 0, sz.skinny_mn);
    P.max_kn_items = sz.kn_items;
    P.max_row_items = sz.row_items;
    P.max_mn = sz.mn;
    P.max_mn_items = sz.mn_items;
    P.any_cm = compact && sz.cm;
    P.max_col_tag = sz.col_tag;
    P.any_conv_n = compact && sz.conv_n;
    P.max_conv_items = sz.conv_items;
    P.flags = (check ? F_CHECK : 0) | (compact ? F_COMPACT : F_SPDZ);
    // cvec sums, check accumulators, and [Z]_p = [C]_p ([tZ]_p = [tC]_p) of
    // skinny layers, all accumulated into atomically by the passes
    P.zero_what = (compact ? 1 : 0) | (check ? 2 : 0) | (sz.skinny ? 4 : 0) | (sz.skinny && !compact ? 8 : 0);
    for (int l = 0; l < n; l++) {
        const int64_t N = L[l].N;
        const int v = N > SKINNY_MAX_N ? 0 : (N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : SKINNY_MAX_N)));
        P.variants |= 1 << (compact && CT_COMPRESS_ALONG_M(L[l].M, N, L[l].compress) ? VARIANT_CM + v : v);
    }
    return CT_OK;
}

// Whether a prepared two-party online call can run as the persistent launch:
// it carries the fused check and all its layers are matrix-core layers (N >
// SKINNY_MAX_N) that are neither convolutions nor compressed along M.
bool persist_ok(const OnlineLaunch &P) {
    return P.check && P.variants == 1 && !P.any_open_u && !P.any_conv_n && !P.any_cm && P.nm > 0;
}

// The kernels of the online phase, in order, on the lane's stream (or, in
// the persistent launch mode, the one persistent launch when the call
// qualifies).
ct_status enqueue_online(ct_ctx *c, Lane &ln, const OnlineLaunch &P) {
    if (c->np > 2) return enqueue_online_np(c, ln, P);
    const int n = P.n;
    if (c->launch_mode == CT_LAUNCH_PERSISTENT && persist_ok(P)) {
        PersistArgs a;
        a.Ls = ln.layers_dev;
        a.jobs = ln.pack_dev;
        a.probs = ln.gemm_dev;
        a.out = P.out_dev;
        a.sync = ln.sync_dev;
        a.wait_ticks = c->launch_wait;
        a.n = n;
        a.flags = P.flags;
        a.zero_what = P.zero_what;
        a.njobs = P.njobs;
        a.pack_tiles = P.pack_tiles;
        a.nprobs = P.nm;
        a.total_tiles = P.total_tiles;
        a.xcd_remap = P.tu.xcd_remap;
        a.any_accum = P.any_accum ? 1 : 0;
        a.mt = ln.gemm_host[0].mt;
        // the launch's counters start at zero (a fill kernel, not a memset,
        // so that the launch can be captured into a graph)
        LAUNCH(c, ln, ST_FILL_ZERO, launch_fill_zero(16, reinterpret_cast<u128 *>(ln.sync_dev), 3, ln.stream));
        LAUNCH(c, ln, ST_PERSIST, launch_online_persist(c->eb, a, c->num_cus, ln.stream));
        return CT_OK;
    }
    if (P.zero_what)
        LAUNCH(c, ln, ST_ZERO_ACC, launch_zero_acc(c->eb, ln.layers_dev, n, P.zero_what, P.max_zero, ln.stream));
    if (P.any_open_u)
        LAUNCH(c, ln, ST_OPEN_U, launch_open_u(c->eb, ln.layers_dev, n, P.flags, P.max_kn_items, ln.stream));
    if (P.open_tiles > 0)
        LAUNCH(c, ln, ST_OPEN_PACK, launch_open_pack(c->eb, ln.layers_dev, n, P.flags, P.open_tiles, ln.stream));
    if (P.any_conv_n)
        LAUNCH(c, ln, ST_CONV_COMPRESS, launch_conv_compress(c->eb, ln.layers_dev, n, P.max_conv_items, ln.stream));
    LAUNCH(c, ln, ST_ROW_PASS, launch_row_pass(c->eb, ln.layers_dev, n, P.flags, P.max_row_items, P.variants, ln.stream));
    if (P.any_cm) LAUNCH(c, ln, ST_COL_TAG, launch_col_tag(c->eb, ln.layers_dev, n, P.max_col_tag, ln.stream));
    if (P.njobs > 0) LAUNCH(c, ln, ST_PACK, launch_pack(c->eb, ln.pack_dev, P.njobs, P.pack_tiles, ln.stream));
    if (P.any_accum)
        LAUNCH(c, ln, ST_COPY_BASE, launch_prob_base(c->eb, ln.gemm_dev, P.nm, P.max_mn, ln.stream));
    ct_status s = run_gemms(c, ln, P.nm, P.total_tiles, P.tu);
    if (s != CT_OK) return s;
    LAUNCH(c, ln, ST_POST, launch_post(c->eb, ln.layers_dev, n, P.flags, P.max_mn_items, ln.stream));
    if (P.compact) LAUNCH(c, ln, ST_COMPACT_FINAL, launch_compact_final(c->eb, ln.layers_dev, n, P.flags, ln.stream));
    if (P.check) LAUNCH(c, ln, ST_FINALIZE, launch_finalize(c->eb, ln.layers_dev, n, P.out_dev, ln.stream));
    return CT_OK;
}

ct_status run_online(ct_ctx *c, Lane &ln, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                     ct_check_result *out_dev) {
    OnlineLaunch P;
    ct_status s = prepare_online(c, ln, mode, L, B, n, out_dev, P);
    return s != CT_OK ? s : enqueue_online(c, ln, P);
}

ct_status prepare_online_split(ct_ctx *c, Lane &a, Lane &b, ct_mode mode, const ct_layer_desc *L,
                               const ct_layer_bufs *B, int n, ct_check_result *out_dev, OnlineLaunch &Pa,
                               OnlineLaunch &Pb, bool &split) {
    split = false;
    if (!c) return CT_EINVAL;
    if (n <= 0 || !L || !B || !b.layers_dev || !c->overlap) return prepare_online(c, a, mode, L, B, n, out_dev, Pa);
    // the whole batch first, so that an error names the caller's layer index
    if (mode != CT_MODE_SPDZ2K && mode != CT_MODE_COMPACT) return fail(c, CT_EINVAL, "unknown mode");
    ct_status v = validate(c, a.max_layers, L, B, n,
                           NEED_INPUTS | NEED_TRIPLE | NEED_OUT | NEED_WORK |
                               (mode == CT_MODE_COMPACT ? NEED_CVEC : 0));
    if (v != CT_OK) return v;
    std::vector<int> ia, ib;
    for (int l = 0; l < n; l++) (L[l].N > SKINNY_MAX_N ? ib : ia).push_back(l);
    if (ia.empty() || ib.empty()) return prepare_online(c, a, mode, L, B, n, out_dev, Pa);
    std::vector<ct_layer_desc> La, Lb;
    std::vector<ct_layer_bufs> Ba, Bb;
    for (int l : ia) { La.push_back(L[l]); Ba.push_back(B[l]); }
    for (int l : ib) { Lb.push_back(L[l]); Bb.push_back(B[l]); }
    ct_status s = prepare_online(c, b, mode, Lb.data(), Bb.data(), (int)ib.size(), out_dev, Pb, ib.data());
    if (s == CT_OK) s = prepare_online(c, a, mode, La.data(), Ba.data(), (int)ia.size(), out_dev, Pa, ia.data());
    split = s == CT_OK;
    return s;
}

ct_status enqueue_online_split(ct_ctx *c, Lane &a, Lane &b, hipEvent_t fork, hipEvent_t join, const OnlineLaunch &Pa,
                               const OnlineLaunch &Pb, bool split) {
    if (!split) return enqueue_online(c, a, Pa);
    // lane b starts after what the caller enqueued on lane a so far
    HIPCHK(c, hipEventRecord(fork, a.stream));
    HIPCHK(c, hipStreamWaitEvent(b.stream, fork, 0));
    ct_status s = enqueue_online(c, b, Pb);
    if (s == CT_OK) s = enqueue_online(c, a, Pa);
    // and lane a's later work after lane b's (also on failure, so that the
    // streams stay joined)
    HIPCHK(c, hipEventRecord(join, b.stream));
    HIPCHK(c, hipStreamWaitEvent(a.stream, join, 0));
    return s;
}

ct_status run_check(ct_ctx *c, Lane &ln, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                    ct_check_result *out_dev) {
    if (!c) return CT_EINVAL;
    if (mode != CT_MODE_SPDZ2K && mode != CT_MODE_COMPACT) return fail(c, CT_EINVAL, "unknown mode");
    const bool compact = mode == CT_MODE_COMPACT;
    ct_status s = validate(c, ln.max_layers, L, B, n, NEED_INPUTS | NEED_TRIPLE | NEED_OUT | (compact ? NEED_CVEC : 0));
    if (s != CT_OK) return s;
    if (!aligned16(out_dev)) return fail(c, CT_EINVAL, "out_dev is null or misaligned");
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = stage_layers(c, ln, L, B, n)) != CT_OK) return s;
    if ((s = upload(c, ln, n, 0)) != CT_OK) return s;
    const Sizes sz = max_sizes(L, n);
    const int mask = compact ? 0x3 : 0x7;
    if (c->np > 2) {
        LAUNCH(c, ln, ST_ZERO_ACC, launch_np_zero(c->eb, ln.layers_dev, n, 2, 0, ln.stream));
        LAUNCH(c, ln, ST_CHECK_BATCH,
               launch_np_check_batch(c->eb, ln.layers_dev, n, mask, std::max({sz.mk, sz.nr, sz.mn}), ln.stream));
        if (compact) LAUNCH(c, ln, ST_CHECK_COMPACT, launch_np_check_compact(c->eb, ln.layers_dev, n, ln.stream));
        LAUNCH(c, ln, ST_FINALIZE, launch_np_finalize(c->eb, ln.layers_dev, n, out_dev, ln.stream));
        return CT_OK;
    }
    LAUNCH(c, ln, ST_ZERO_ACC, launch_zero_acc(c->eb, ln.layers_dev, n, 2, 0, ln.stream));
    LAUNCH(c, ln, ST_CHECK_BATCH,
           launch_check_batch(c->eb, ln.layers_dev, n, mask, std::max({sz.mk, sz.nr, sz.mn}), ln.stream));
    if (compact) LAUNCH(c, ln, ST_CHECK_COMPACT, launch_check_compact(c->eb, ln.layers_dev, n, ln.stream));
    LAUNCH(c, ln, ST_FINALIZE, launch_finalize(c->eb, ln.layers_dev, n, out_dev, ln.stream));
    return CT_OK;
}

}  // namespace ct

extern "C" {

ct_status ct_tag_linear(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n) {
    if (!c) return CT_EINVAL;
    return run_online(c, c->main, mode, L, B, n, nullptr);
}

ct_status ct_tag_linear_check(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                              ct_check_result *out_dev) {
    if (!c) return CT_EINVAL;
    if (!out_dev) return fail(c, CT_EINVAL, "null result array");
    // with per-launch timing on, every stage runs once over the whole batch
    // on the main lane, so that each stage's time covers all layers
    if (c->timing) return run_online(c, c->main, mode, L, B, n, out_dev);
    OnlineLaunch Pa, Pb;
    bool split = false;
    ct_status s = prepare_online_split(c, c->main, c->side, mode, L, B, n, out_dev, Pa, Pb, split);
    return s != CT_OK ? s : enqueue_online_split(c, c->main, c->side, c->fork, c->join, Pa, Pb, split);
}

ct_status ct_tag_linear_check_static(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B,
                                     int n, ct_check_result *out_dev) {
    if (!c) return CT_EINVAL;
    if (!L || !B) return fail(c, CT_EINVAL, "null layer or buffer array");
    if (n < 1 || n > (int)c->static_bufs.size())
        return fail(c, CT_EINVAL, "n must be in [1, max_layers] (" + std::to_string(c->static_bufs.size()) + ")");
    if (!c->static_work) return fail(c, CT_EDEVICE, "no static workspace on this device");
    // the layers' workspaces, one after another at 256-byte boundaries
    const int64_t cap = CT_STATIC_WORK_BYTES;
    int64_t off = 0;
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        ct_layer_bufs &b = c->static_bufs[l];
        b = B[l];
        b.work = nullptr;
        if (d.N <= SKINNY_MAX_N) continue;  // no workspace
        // M, K, N of any size are rejected before their products could overflow
        if (d.M < 1 || d.K < 1 || d.N < 1 || d.M * d.K > cap || d.N * d.K > cap)
            return fail(c, CT_EINVAL, "layer " + std::to_string(l) + ": needs more workspace than the static "
                                      "workspace holds (" + std::to_string(cap) + " bytes)");
        const int64_t bytes = (int64_t)CT_WORK_LEN_NP(d.M, d.K, d.N, (int64_t)c->np) * c->eb;
        off = (off + 255) & ~(int64_t)255;
        if (bytes > cap - off)
            return fail(c, CT_EINVAL, "layers 0.." + std::to_string(l) + " need more than the " + std::to_string(cap) +
                                      " bytes of the static workspace (CT_STATIC_WORK_BYTES)");
        b.work = reinterpret_cast<ct_u128 *>(static_cast<uint8_t *>(c->static_work) + off);
        off += bytes;
    }
    return ct_tag_linear_check(c, mode, L, c->static_bufs.data(), n, out_dev);
}

ct_status ct_mac_check_device(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                              ct_check_result *out_dev) {
    if (!c) return CT_EINVAL;
    return run_check(c, c->main, mode, L, B, n, out_dev);
}

ct_status ct_mac_check(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                       ct_check_result *out) {
    if (!c) return CT_EINVAL;
    if (!out) return fail(c, CT_EINVAL, "null result array");
    Lane &ln = c->main;
    ct_status s = run_check(c, ln, mode, L, B, n, ln.res_dev);
    if (s != CT_OK) return s;
    HIPCHK(c, hipMemcpyAsync(ln.res_host, ln.res_dev, sizeof(ct_check_result) * n, hipMemcpyDeviceToHost, ln.stream));
    HIPCHK(c, hipStreamSynchronize(ln.stream));
    bool ok = true;
    for (int l = 0; l < n; l++) {
        out[l] = ln.res_host[l];
        ok = ok && ln.res_host[l].accept;
    }
    return ok ? CT_OK : CT_ABORT;
}

ct_status ct_plan_create(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                         ct_check_result *out_dev, ct_plan **out) {
    if (!c || !out) return CT_EINVAL;
    *out = nullptr;
    HIPCHK(c, hipSetDevice(c->device));
    ct_plan *pl = new ct_plan();
    pl->ctx = c;
    hipStream_t st = nullptr, side = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = lane_init(pl->lane, st, std::max(n, 1));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
    if (e == hipSuccess) e = lane_init(pl->side, side, std::max(n, 1));
    else pl->side.stream = side;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join, hipEventDisableTiming);
    if (e != hipSuccess) {
        ct_plan_destroy(pl);
        return hip_fail(c, e, "ct_plan_create");
    }
    OnlineLaunch Pa, Pb;
    bool split = false;
    ct_status s = prepare_online_split(c, pl->lane, pl->side, mode, L, B, n, out_dev, Pa, Pb, split);
    if (s == CT_OK) {
        // the tables are uploaded before the capture starts, so the graph
        // holds kernel nodes only; the side stream joins the capture through
        // the fork event and is joined back before it ends
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamSynchronize(side);
        if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            s = enqueue_online_split(c, pl->lane, pl->side, pl->fork, pl->join, Pa, Pb, split);
            const hipError_t e2 = hipStreamEndCapture(st, &pl->graph);
            if (s == CT_OK && e2 != hipSuccess) e = e2;
        }
        if (s == CT_OK && e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
        if (s == CT_OK && e != hipSuccess) s = hip_fail(c, e, "graph capture");
    }
    if (s != CT_OK) {
        ct_plan_destroy(pl);
        return s;
    }
    *out = pl;
    return CT_OK;
}

ct_status ct_plan_launch(ct_plan *pl) {
    if (!pl) return CT_EINVAL;
    ct_ctx *c = pl->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipGraphLaunch(pl->exec, c->main.stream));
    return CT_OK;
}

ct_status ct_plan_destroy(ct_plan *pl) {
    if (!pl) return CT_EINVAL;
    (void)hipSetDevice(pl->ctx->device);
    if (pl->lane.stream) (void)hipStreamSynchronize(pl->lane.stream);
    // a replay may still be running on the context stream
    (void)hipStreamSynchronize(pl->ctx->main.stream);
    if (pl->side.stream) (void)hipStreamSynchronize(pl->side.stream);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->fork) (void)hipEventDestroy(pl->fork);
    if (pl->join) (void)hipEventDestroy(pl->join);
    hipStream_t st = pl->lane.stream, side = pl->side.stream;
    lane_free(pl->lane);
    lane_free(pl->side);
    if (st) (void)hipStreamDestroy(st);
    if (side) (void)hipStreamDestroy(side);
    delete pl;
    return CT_OK;
}

ct_status ct_set_overlap(ct_ctx *c, int enable) {
    if (!c) return CT_EINVAL;
    c->overlap = enable != 0;
    return CT_OK;
}

ct_status ct_set_launch(ct_ctx *c, int mode) {
    if (!c) return CT_EINVAL;
    if (mode != CT_LAUNCH_STAGED && mode != CT_LAUNCH_PERSISTENT) return fail(c, CT_EINVAL, "unknown launch mode");
    c->launch_mode = mode;
    return CT_OK;
}

ct_status ct_set_launch_wait(ct_ctx *c, uint64_t ticks) {
    if (!c) return CT_EINVAL;
    c->launch_wait = ticks;
    return CT_OK;
}

ct_status ct_set_timing(ct_ctx *c, int enable) {
    if (!c) return CT_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    if (enable && c->ev_start.empty()) {
        c->ev_start.resize(EV_POOL);
        c->ev_end.resize(EV_POOL);
        c->ev_stage.resize(EV_POOL);
        for (int i = 0; i < EV_POOL; i++) {
            HIPCHK(c, hipEventCreate(&c->ev_start[i]));
            HIPCHK(c, hipEventCreate(&c->ev_end[i]));
        }
    }
    if (!enable) HIPCHK(c, fold_timing(c));
    c->timing = enable != 0;
    return CT_OK;
}

ct_status ct_set_tuning(ct_ctx *c, const ct_tuning *t) {
    if (!c || !t) return CT_EINVAL;
    if (t->group_m < 1 || t->split_target < 0 || t->split_target > MAX_STEPS_PER_SPLIT || t->xcd_remap < 0 ||
        t->xcd_remap > 4096 || t->tile < CT_TILE_AUTO || t->tile > CT_TILE_REGS_FIT)
        return fail(c, CT_EINVAL, "invalid tuning");
    c->fallback = GemmTuning{t->group_m, t->xcd_remap, t->split_target, t->tile};
    c->tuned.clear();
    return CT_OK;
}

ct_status ct_get_tuning(const ct_ctx *c, ct_mode mode, const ct_layer_desc *L, int n, ct_tuning *out) {
    if (!c || !L || !out || n < 1) return CT_EINVAL;
    const GemmTuning t = tuning_for(c, shape_class(mode, L, n));
    out->group_m = t.group_m;
    out->xcd_remap = t.xcd_remap;
    out->split_target = t.split_target;
    out->tile = t.tile;
    out->gemm_ms = -1.0;
    return CT_OK;
}

ct_status ct_autotune(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n, int reps,
                      ct_tuning *best_out) {
    if (!c) return CT_EINVAL;
    if (reps < 1) reps = 1;
    const bool was_timing = c->timing;
    ct_status s = ct_set_timing(c, 1);
    if (s != CT_OK) return s;
    HIPCHK(c, fold_timing(c));
    // the trials' stage times are not the caller's: restored afterwards
    double saved_ms[ST_COUNT];
    int64_t saved_n[ST_COUNT];
    std::copy(c->stage_ms, c->stage_ms + ST_COUNT, saved_ms);
    std::copy(c->stage_n, c->stage_n + ST_COUNT, saved_n);
    static const int groups[] = {1, 2, 4, 8, 16, 64};
    static const int splits[] = {0, 16, 32, 64, 128};
    static const int remaps[] = {0, 1, 4, 8, 16};
    static const int tiles64[] = {CT_TILE_LDS_64x64, CT_TILE_REGS_64x64, CT_TILE_REGS_FIT};
    static const int tiles32[] = {CT_TILE_LDS_64x64, CT_TILE_REGS_64x64, CT_TILE_REGS_FIT, CT_TILE_LDS_128x64,
                                  CT_TILE_REGS_128x64};
    GemmTuning best = c->fallback;
    if (best.tile == CT_TILE_AUTO) best.tile = CT_TILE_REGS_64x64;
    double best_ms = 1e30;
    // times the products under one candidate (with the copy of the constant
    // terms that split products need first); keeps it if it is the fastest
    auto trial = [&](const GemmTuning &cand) -> ct_status {
        c->forcing = true;
        c->forced = cand;
        ct_status st = run_online(c, c->main, mode, L, B, n, nullptr);  // warm-up
        if (st == CT_OK) {
            HIPCHK(c, fold_timing(c));
            for (int k : {ST_RING_GEMM, ST_COPY_BASE}) c->stage_ms[k] = 0, c->stage_n[k] = 0;
            for (int r = 0; r < reps && st == CT_OK; r++) st = run_online(c, c->main, mode, L, B, n, nullptr);
        }
        if (st == CT_OK) {
            HIPCHK(c, fold_timing(c));
            const double ms = (c->stage_ms[ST_RING_GEMM] + c->stage_ms[ST_COPY_BASE]) / reps;
            if (c->stage_n[ST_RING_GEMM] > 0 && ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
        c->forcing = false;
        return st;
    };
    // coordinate descent from the current configuration: the kernel and
    // workgroup tile shape, the K split, the XCD mapping, the tile order;
    // then the tile shape once more under the chosen rest
    const int *tl = c->eb == 8 ? tiles32 : tiles64;
    const int ntl = c->eb == 8 ? 5 : 3;
    s = trial(best);
    for (int pass = 0; pass < 2 && s == CT_OK; pass++) {
        for (int i = 0; i < ntl && s == CT_OK; i++)
            if (tl[i] != best.tile) { GemmTuning t = best; t.tile = tl[i]; s = trial(t); }
        if (pass == 1) break;
        for (int sp : splits)
            if (s == CT_OK && sp != best.split_target) { GemmTuning t = best; t.split_target = sp; s = trial(t); }
        for (int xcd : remaps)
            if (s == CT_OK && xcd != best.xcd_remap) { GemmTuning t = best; t.xcd_remap = xcd; s = trial(t); }
        for (int g : groups)
            if (s == CT_OK && g != best.group_m) { GemmTuning t = best; t.group_m = g; s = trial(t); }
    }
    std::copy(saved_ms, saved_ms + ST_COUNT, c->stage_ms);
    std::copy(saved_n, saved_n + ST_COUNT, c->stage_n);
    if (s != CT_OK) return s;
    if (!was_timing) {
        c->timing = false;
    }
    c->tuned[shape_class(mode, L, n)] = best;
    if (best_out) {
        best_out->group_m = best.group_m;
        best_out->xcd_remap = best.xcd_remap;
        best_out->split_target = best.split_target;
        best_out->tile = best.tile;
        best_out->gemm_ms = best_ms < 1e29 ? best_ms : -1.0;
    }
    return CT_OK;
}

ct_status ct_stage_times(ct_ctx *c, ct_stage_time *out, int max, int *count) {
    if (!c || !count || (max > 0 && !out)) return CT_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, fold_timing(c));
    int k = 0;
    for (int st = 0; st < ST_COUNT; st++) {
        if (c->stage_n[st] == 0) continue;
        if (k < max) {
            std::snprintf(out[k].name, sizeof(out[k].name), "%s", kStageNames[st]);
            out[k].total_ms = c->stage_ms[st];
            out[k].launches = c->stage_n[st];
        }
        k++;
        c->stage_ms[st] = 0;
        c->stage_n[st] = 0;
    }
    *count = k;
    return CT_OK;
}

}  // extern "C"
