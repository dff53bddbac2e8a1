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
#include <string>
#include <unordered_map>
#include <vector>

#include "compacttag.h"
#include "ct_internal.h"

using namespace ct;

// Kernel stages, for the optional per-launch timing (ct_set_timing).
enum Stage : int {
    ST_DEAL_LIFT, ST_FILL_ZERO, ST_DEAL_AUTH, ST_DEAL_SKINNY, ST_ZERO_ACC, ST_OPEN_U, ST_ROW_PASS, ST_PACK,
    ST_COPY_BASE, ST_RING_GEMM, ST_POST, ST_COMPACT_FINAL, ST_CHECK_BATCH, ST_CHECK_COMPACT, ST_FINALIZE, ST_COUNT
};
static const char *kStageNames[ST_COUNT] = {
    "deal_lift", "fill_zero", "deal_auth", "deal_skinny", "zero_acc", "open_u", "row_pass", "pack",
    "copy_base", "ring_gemm", "post", "compact_final", "check_batch", "check_compact", "finalize"};
constexpr int EV_POOL = 2048;

struct ct_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t delta[2] = {0, 0};
    int max_layers = 0, max_probs = 0;
    int num_cus = 256;
    LayerDev *layers_dev = nullptr, *layers_host = nullptr;
    GemmProb *gemm_dev = nullptr, *gemm_host = nullptr;
    PackJob *pack_dev = nullptr, *pack_host = nullptr;
    SkinnyProb *skinny_dev = nullptr, *skinny_host = nullptr;
    int max_jobs = 0;
    u128 *acc_dev = nullptr;
    ct_check_result *res_dev = nullptr, *res_host = nullptr;
    hipEvent_t upload_done = nullptr;
    std::string err;
    // per-launch timing: event pairs recorded around each kernel on `stream`
    bool timing = false;
    std::vector<hipEvent_t> ev_start, ev_end;
    std::vector<int> ev_stage;
    int ev_used = 0;
    double stage_ms[ST_COUNT] = {};
    int64_t stage_n[ST_COUNT] = {};
    // launch configuration of the matrix-core products per shape class
    std::unordered_map<uint64_t, GemmTuning> tuned;
    GemmTuning fallback = {1, 0, 0};
    bool forcing = false;
    GemmTuning forced = {1, 0, 0};
};

namespace {

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

ct_status fail(ct_ctx *c, ct_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}
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
    hipError_t e = hipStreamSynchronize(c->stream);
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

// Runs a launcher; with timing on, brackets it with an event pair on the stream.
#define LAUNCH(ctx, stage, expr)                                                         \
    do {                                                                                 \
        if ((ctx)->timing) {                                                             \
            if ((ctx)->ev_used == EV_POOL) HIPCHK(ctx, fold_timing(ctx));                \
            HIPCHK(ctx, hipEventRecord((ctx)->ev_start[(ctx)->ev_used], (ctx)->stream)); \
        }                                                                                \
        HIPCHK(ctx, expr);                                                               \
        if ((ctx)->timing) {                                                             \
            HIPCHK(ctx, hipEventRecord((ctx)->ev_end[(ctx)->ev_used], (ctx)->stream));   \
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

ct_status validate(ct_ctx *c, const ct_layer_desc *L, const ct_layer_bufs *B, int n, unsigned need) {
    if (!c) return CT_EINVAL;
    if (!L || !B) return fail(c, CT_EINVAL, "null layer or buffer array");
    if (n < 1 || n > c->max_layers)
        return fail(c, CT_EINVAL, "n must be in [1, max_layers] (" + std::to_string(c->max_layers) + ")");
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        const std::string at = "layer " + std::to_string(l) + ": ";
        if (d.M < 1 || d.K < 1 || d.N < 1) return fail(c, CT_EINVAL, at + "M, K, N must be >= 1");
        if (d.M >= (1LL << 31) || d.K >= (1LL << 31) || d.N >= (1LL << 31))
            return fail(c, CT_EINVAL, at + "M, K, N must be < 2^31");
        if (d.f != 0) return fail(c, CT_EINVAL, at + "f must be 0 (truncation is not on this path)");
        if (d.layer_id >= (1ULL << 48)) return fail(c, CT_EINVAL, at + "layer_id must be < 2^48");
        const ct_layer_bufs &b = B[l];
        auto chk = [&](const ct_u128 *p, const char *name) -> bool {
            if (!aligned16(p)) {
                c->err = at + "buffer " + name + " is null or not 16-byte aligned";
                return false;
            }
            return true;
        };
        for (int p = 0; p < 2; p++) {
            if (need & NEED_INPUTS)
                if (!chk(b.X[p], "X") || !chk(b.tX[p], "tX") || !chk(b.Y[p], "Y") || !chk(b.tY[p], "tY"))
                    return CT_EINVAL;
            if (need & NEED_TRIPLE)
                if (!chk(b.A[p], "A") || !chk(b.tA[p], "tA") || !chk(b.B[p], "B") || !chk(b.tB[p], "tB") ||
                    !chk(b.C[p], "C") || !chk(b.tC[p], "tC") || !chk(b.R[p], "R") || !chk(b.tR[p], "tR"))
                    return CT_EINVAL;
            if (need & NEED_OUT)
                if (!chk(b.Z[p], "Z") || !chk(b.tZ[p], "tZ")) return CT_EINVAL;
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

void fill_layer(const ct_ctx *c, const ct_layer_desc &d, const ct_layer_bufs &b, int l, LayerDev &o) {
    std::memset(&o, 0, sizeof(o));
    o.M = d.M;
    o.K = d.K;
    o.N = d.N;
    o.delta[0] = c->delta[0];
    o.delta[1] = c->delta[1];
    const uint64_t s = d.seed, id = d.layer_id;
    o.key[K_LIFT_X] = hkey(s, id, P_LIFT_X);
    o.key[K_LIFT_Y] = hkey(s, id, P_LIFT_Y);
    o.key[K_LIFT_A] = hkey(s, id, P_LIFT_A);
    o.key[K_LIFT_B] = hkey(s, id, P_LIFT_B);
    o.key[K_LIFT_R] = hkey(s, id, P_LIFT_R);
    for (int obj = 1; obj <= 6; obj++) {
        o.key[K_VSH_X + obj - 1] = hkey(s, id, P_VSH + obj);
        o.key[K_TSH_X + obj - 1] = hkey(s, id, P_TSH + obj);
    }
    o.key[K_CHI] = hkey(s, id, P_CHI);
    o.key[K_CHIHAT] = hkey(s, id, P_CHIHAT);
    o.key[K_CHI_E] = hkey(s, id, P_CHI_E);
    o.key[K_CHI_U] = hkey(s, id, P_CHI_U);
    o.key[K_CHI_D] = hkey(s, id, P_CHI_D);
    auto cp = [](u128 *dst[2], ct_u128 *const src[2]) {
        dst[0] = reinterpret_cast<u128 *>(src[0]);
        dst[1] = reinterpret_cast<u128 *>(src[1]);
    };
    cp(o.X, b.X); cp(o.tX, b.tX); cp(o.A, b.A); cp(o.tA, b.tA);
    cp(o.Y, b.Y); cp(o.tY, b.tY); cp(o.B, b.B); cp(o.tB, b.tB);
    cp(o.C, b.C); cp(o.tC, b.tC); cp(o.R, b.R); cp(o.tR, b.tR);
    cp(o.Z, b.Z); cp(o.tZ, b.tZ);
    o.E = reinterpret_cast<u128 *>(b.E);
    o.U = reinterpret_cast<u128 *>(b.U);
    o.D = reinterpret_cast<u128 *>(b.D);
    o.cvec = reinterpret_cast<u128 *>(b.cvec);
    o.work = reinterpret_cast<u128 *>(b.work);
    o.acc = c->acc_dev + (size_t)l * ACC_PER_LAYER;
}

struct Sizes {
    int64_t mk = 0, kn = 0, mn = 0, m = 0, k = 0, cvec = 0, kn_items = 0, mn_items = 0;
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
        s.cvec = std::max(s.cvec, (int64_t)CT_CVEC_LEN(d.M, d.K));
        s.kn_items = std::max(s.kn_items, sweep_items(d.K, d.N));
        s.mn_items = std::max(s.mn_items, sweep_items(d.M, d.N));
    }
    return s;
}

// Waits for the previous upload, then stages layers (and GEMM problems).
ct_status stage_layers(ct_ctx *c, const ct_layer_desc *L, const ct_layer_bufs *B, int n) {
    HIPCHK(c, hipEventSynchronize(c->upload_done));
    for (int l = 0; l < n; l++) fill_layer(c, L[l], B[l], l, c->layers_host[l]);
    return CT_OK;
}

ct_status upload(ct_ctx *c, int n, int nprobs, int njobs = 0, int nskinny = 0) {
    HIPCHK(c, hipMemcpyAsync(c->layers_dev, c->layers_host, sizeof(LayerDev) * n, hipMemcpyHostToDevice,
                             c->stream));
    if (nprobs > 0)
        HIPCHK(c, hipMemcpyAsync(c->gemm_dev, c->gemm_host, sizeof(GemmProb) * nprobs, hipMemcpyHostToDevice,
                                 c->stream));
    if (njobs > 0)
        HIPCHK(c, hipMemcpyAsync(c->pack_dev, c->pack_host, sizeof(PackJob) * njobs, hipMemcpyHostToDevice,
                                 c->stream));
    if (nskinny > 0)
        HIPCHK(c, hipMemcpyAsync(c->skinny_dev, c->skinny_host, sizeof(SkinnyProb) * nskinny,
                                 hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipEventRecord(c->upload_done, c->stream));
    return CT_OK;
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

PackJob make_job(const u128 *src, u128 *dst, int64_t rows, int64_t cols, int side) {
    PackJob j;
    std::memset(&j, 0, sizeof(j));
    j.src = src; j.dst = dst; j.rows = (int32_t)rows; j.cols = (int32_t)cols; j.side = side;
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
int plan_gemms(std::vector<GemmProb> &probs, int num_cus, const GemmTuning &tu, int *total_tiles, bool *any_accum) {
    int64_t total_steps = 0;
    for (auto &p : probs) {
        p.tiles_m = (p.M + 63) / 64;
        p.tiles_n = (p.N + 63) / 64;
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

ct_status run_gemms(ct_ctx *c, int nprobs, int total_tiles, const GemmTuning &tu) {
    if (nprobs > 0) LAUNCH(c, ST_RING_GEMM, launch_gemm(c->gemm_dev, nprobs, total_tiles, tu.xcd_remap, c->stream));
    return CT_OK;
}

}  // namespace

extern "C" {

ct_status ct_create(ct_ctx **out, const ct_params *p) {
    if (!out || !p) return CT_EINVAL;
    *out = nullptr;
    if (p->k_bits != 64 || p->s_bits != 64) return CT_EINVAL;
    ct_ctx *c = new ct_ctx();
    c->device = p->device;
    c->stream = reinterpret_cast<hipStream_t>(p->hip_stream);
    c->max_layers = p->max_layers > 0 ? p->max_layers : 256;
    c->max_probs = 4 * c->max_layers;
    c->max_jobs = 10 * c->max_layers;
    for (int q = 0; q < 2; q++) c->delta[q] = hdraw(hkey(p->key_seed, GLOBAL_LAYER, P_KEY + q), 0);
    auto bail = [&](hipError_t e, const char *what) {
        std::fprintf(stderr, "ct_create: %s: %s\n", what, hipGetErrorString(e));
        ct_destroy(c);
        return CT_EDEVICE;
    };
    hipError_t e;
    if ((e = hipSetDevice(c->device)) != hipSuccess) return bail(e, "hipSetDevice");
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
        c->num_cus = cus;
    if ((e = hipMalloc(&c->layers_dev, sizeof(LayerDev) * c->max_layers)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = hipMalloc(&c->gemm_dev, sizeof(GemmProb) * c->max_probs)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = hipMalloc(&c->pack_dev, sizeof(PackJob) * c->max_jobs)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = hipMalloc(&c->skinny_dev, sizeof(SkinnyProb) * c->max_layers)) != hipSuccess)
        return bail(e, "hipMalloc");
    if ((e = hipHostMalloc(&c->pack_host, sizeof(PackJob) * c->max_jobs, hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = hipHostMalloc(&c->skinny_host, sizeof(SkinnyProb) * c->max_layers, hipHostMallocDefault)) !=
        hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = hipMalloc(&c->acc_dev, sizeof(u128) * ACC_PER_LAYER * c->max_layers)) != hipSuccess)
        return bail(e, "hipMalloc");
    if ((e = hipMalloc(&c->res_dev, sizeof(ct_check_result) * c->max_layers)) != hipSuccess)
        return bail(e, "hipMalloc");
    if ((e = hipHostMalloc(&c->layers_host, sizeof(LayerDev) * c->max_layers, hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = hipHostMalloc(&c->gemm_host, sizeof(GemmProb) * c->max_probs, hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = hipHostMalloc(&c->res_host, sizeof(ct_check_result) * c->max_layers, hipHostMallocDefault)) !=
        hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming)) != hipSuccess)
        return bail(e, "hipEventCreate");
    if ((e = hipEventRecord(c->upload_done, c->stream)) != hipSuccess) return bail(e, "hipEventRecord");
    *out = c;
    return CT_OK;
}

ct_status ct_destroy(ct_ctx *c) {
    if (!c) return CT_EINVAL;
    if (c->stream || c->layers_dev) hipStreamSynchronize(c->stream);
    if (c->upload_done) hipEventDestroy(c->upload_done);
    for (auto e : c->ev_start) hipEventDestroy(e);
    for (auto e : c->ev_end) hipEventDestroy(e);
    if (c->layers_dev) hipFree(c->layers_dev);
    if (c->gemm_dev) hipFree(c->gemm_dev);
    if (c->acc_dev) hipFree(c->acc_dev);
    if (c->pack_dev) hipFree(c->pack_dev);
    if (c->skinny_dev) hipFree(c->skinny_dev);
    if (c->pack_host) hipHostFree(c->pack_host);
    if (c->skinny_host) hipHostFree(c->skinny_host);
    if (c->res_dev) hipFree(c->res_dev);
    if (c->layers_host) hipHostFree(c->layers_host);
    if (c->gemm_host) hipHostFree(c->gemm_host);
    if (c->res_host) hipHostFree(c->res_host);
    delete c;
    return CT_OK;
}

ct_status ct_key_shares(const ct_ctx *c, uint64_t out[2]) {
    if (!c || !out) return CT_EINVAL;
    out[0] = c->delta[0];
    out[1] = c->delta[1];
    return CT_OK;
}

const char *ct_last_error(const ct_ctx *c) { return c ? c->err.c_str() : "null context"; }

ct_status ct_gen_triple_tags(ct_ctx *c, const ct_layer_desc *L, const ct_layer_bufs *B, int n, int with_inputs) {
    ct_status s = validate(c, L, B, n, NEED_TRIPLE | NEED_WORK | (with_inputs ? NEED_INPUTS : 0));
    if (s != CT_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = stage_layers(c, L, B, n)) != CT_OK) return s;
    // C~ = A~ B~ with the lifts left in party 1's buffers: packed matrix-core
    // product for wide layers (operand tiles in the workspace), VALU rows for
    // layers with N <= SKINNY_MAX_N.
    std::vector<GemmProb> probs;
    int njobs = 0, nskinny = 0;
    for (int l = 0; l < n; l++) {
        const LayerDev &o = c->layers_host[l];
        const ct_layer_desc &d = L[l];
        if (d.N <= SKINNY_MAX_N) {
            SkinnyProb sp;
            std::memset(&sp, 0, sizeof(sp));
            sp.L = o.A[1]; sp.R = o.B[1]; sp.out = o.C[1];
            sp.M = (int32_t)d.M; sp.N = (int32_t)d.N; sp.K = (int32_t)d.K;
            c->skinny_host[nskinny++] = sp;
            continue;
        }
        const WorkOff w = work_off(d.M, d.K, d.N);
        c->pack_host[njobs++] = make_job(o.A[1], o.work + w.Ep, d.M, d.K, 0);
        c->pack_host[njobs++] = make_job(o.B[1], o.work + w.B0p, d.K, d.N, 1);
        probs.push_back(make_prob(o.work + w.Ep, nullptr, o.work + w.B0p, nullptr, nullptr, o.C[1], d));
    }
    const int pack_tiles = plan_jobs(c->pack_host, njobs);
    int total_tiles = 0;
    bool any_accum = false;
    const GemmTuning tu = c->fallback;
    const int nm = plan_gemms(probs, c->num_cus, tu, &total_tiles, &any_accum);
    std::copy(probs.begin(), probs.end(), c->gemm_host);
    if ((s = upload(c, n, nm, njobs, nskinny)) != CT_OK) return s;
    const Sizes sz = max_sizes(L, n);
    LAUNCH(c, ST_DEAL_LIFT, launch_deal_lift(c->layers_dev, n, std::max(sz.mk, sz.kn), c->stream));
    LAUNCH(c, ST_PACK, launch_pack(c->pack_dev, njobs, pack_tiles, c->stream));
    for (int i = 0; i < nm; i++)
        if (probs[i].accumulate)
            LAUNCH(c, ST_FILL_ZERO, launch_fill_zero(probs[i].out, (int64_t)probs[i].M * probs[i].N, c->stream));
    if ((s = run_gemms(c, nm, total_tiles, tu)) != CT_OK) return s;
    if (nskinny > 0) {
        int max_rows = 0;
        for (int i = 0; i < nskinny; i++) max_rows = std::max(max_rows, c->skinny_host[i].M);
        LAUNCH(c, ST_DEAL_SKINNY, launch_skinny(c->skinny_dev, nskinny, max_rows, c->stream));
    }
    const int mask = (with_inputs ? ((1 << OBJ_X) | (1 << OBJ_Y)) : 0) | (1 << OBJ_A) | (1 << OBJ_B) |
                     (1 << OBJ_C) | (1 << OBJ_R);
    LAUNCH(c, ST_DEAL_AUTH, launch_deal_auth(c->layers_dev, n, mask, std::max({sz.mk, sz.kn, sz.mn}), c->stream));
    return CT_OK;
}

}  // extern "C"

namespace {

// The online phase, optionally with the verification fused into its passes
// (out_dev != nullptr).
ct_status online(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                 ct_check_result *out_dev) {
    if (!c) return CT_EINVAL;
    if (mode != CT_MODE_SPDZ2K && mode != CT_MODE_COMPACT) return fail(c, CT_EINVAL, "unknown mode");
    const bool compact = mode == CT_MODE_COMPACT;
    const bool check = out_dev != nullptr;
    ct_status s = validate(c, L, B, n, NEED_INPUTS | NEED_TRIPLE | NEED_OUT | NEED_WORK | (compact ? NEED_CVEC : 0));
    if (s != CT_OK) return s;
    if (check && !aligned16(out_dev)) return fail(c, CT_EINVAL, "out_dev is null or misaligned");
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = stage_layers(c, L, B, n)) != CT_OK) return s;

    // Matrix-core products (layers with N > SKINNY_MAX_N), both parties,
    // Eq. (2) with E U folded into party 0's left operand by the row pass:
    //   [Z]_0 = [C]_0 + E [B]_0 + (A_0 + E) U,   [Z]_1 = [C]_1 + E [B]_1 + [A]_1 U;
    // SPDZ2k tags of Eq. (3):  [tZ]_p = [tC]_p + E [tB]_p + ([tA]_p + [Delta]_p E) U.
    // Every operand is converted once into digit tiles in the workspace.
    std::vector<GemmProb> probs;
    probs.reserve(4 * n);
    int njobs = 0;
    for (int l = 0; l < n; l++) {
        const ct_layer_desc &d = L[l];
        if (d.N <= SKINNY_MAX_N) continue;
        const LayerDev &o = c->layers_host[l];
        const WorkOff w = work_off(d.M, d.K, d.N);
        u128 *W = o.work;
        PackJob *J = c->pack_host;
        J[njobs++] = make_job(o.E, W + w.Ep, d.M, d.K, 0);
        J[njobs++] = make_job(W + w.AE0, W + w.AE0p, d.M, d.K, 0);
        J[njobs++] = make_job(o.A[1], W + w.A1p, d.M, d.K, 0);
        J[njobs++] = make_job(o.B[0], W + w.B0p, d.K, d.N, 1);
        J[njobs++] = make_job(o.B[1], W + w.B1p, d.K, d.N, 1);
        J[njobs++] = make_job(o.U, W + w.Up, d.K, d.N, 1);
        const size_t first = probs.size();
        probs.push_back(make_prob(W + w.Ep, W + w.AE0p, W + w.B0p, W + w.Up, o.C[0], o.Z[0], d));
        probs.push_back(make_prob(W + w.Ep, W + w.A1p, W + w.B1p, W + w.Up, o.C[1], o.Z[1], d));
        if (!compact) {
            J[njobs++] = make_job(W + w.tAE0, W + w.tAE0p, d.M, d.K, 0);
            J[njobs++] = make_job(W + w.tAE1, W + w.tAE1p, d.M, d.K, 0);
            J[njobs++] = make_job(o.tB[0], W + w.tB0p, d.K, d.N, 1);
            J[njobs++] = make_job(o.tB[1], W + w.tB1p, d.K, d.N, 1);
            probs.push_back(make_prob(W + w.Ep, W + w.tAE0p, W + w.tB0p, W + w.Up, o.tC[0], o.tZ[0], d));
            probs.push_back(make_prob(W + w.Ep, W + w.tAE1p, W + w.tB1p, W + w.Up, o.tC[1], o.tZ[1], d));
        }
        for (size_t j = first; j < probs.size(); j++) probs[j].gsize = (int32_t)(probs.size() - first);
    }
    const int pack_tiles = plan_jobs(c->pack_host, njobs);
    int total_tiles = 0;
    bool any_accum = false;
    const GemmTuning tu = tuning_for(c, shape_class(mode, L, n));
    const int nm = plan_gemms(probs, c->num_cus, tu, &total_tiles, &any_accum);
    std::copy(probs.begin(), probs.end(), c->gemm_host);
    if ((s = upload(c, n, nm, njobs)) != CT_OK) return s;

    const Sizes sz = max_sizes(L, n);
    const int flags = (check ? F_CHECK : 0) | (compact ? F_COMPACT : F_SPDZ);
    const int zero_what = (compact ? 1 : 0) | (check ? 2 : 0);
    if (zero_what) LAUNCH(c, ST_ZERO_ACC, launch_zero_acc(c->layers_dev, n, zero_what, sz.cvec, c->stream));
    LAUNCH(c, ST_OPEN_U, launch_open_u(c->layers_dev, n, flags, sz.kn_items, c->stream));
    int variants = 0;
    for (int l = 0; l < n; l++) {
        const int64_t N = L[l].N;
        variants |= 1 << (N > SKINNY_MAX_N ? 0 : (N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : SKINNY_MAX_N))));
    }
    LAUNCH(c, ST_ROW_PASS, launch_row_pass(c->layers_dev, n, flags, sz.m, variants, c->stream));
    if (njobs > 0) LAUNCH(c, ST_PACK, launch_pack(c->pack_dev, njobs, pack_tiles, c->stream));
    if (any_accum) LAUNCH(c, ST_COPY_BASE, launch_copy_base(c->layers_dev, n, mode, sz.mn, c->stream));
    if ((s = run_gemms(c, nm, total_tiles, tu)) != CT_OK) return s;
    LAUNCH(c, ST_POST, launch_post(c->layers_dev, n, flags, sz.mn_items, c->stream));
    if (compact) LAUNCH(c, ST_COMPACT_FINAL, launch_compact_final(c->layers_dev, n, flags, c->stream));
    if (check) LAUNCH(c, ST_FINALIZE, launch_finalize(c->layers_dev, n, out_dev, c->stream));
    return CT_OK;
}

}  // namespace

extern "C" {

ct_status ct_tag_linear(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n) {
    return online(c, mode, L, B, n, nullptr);
}

ct_status ct_tag_linear_check(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                              ct_check_result *out_dev) {
    if (c && !out_dev) return fail(c, CT_EINVAL, "null result array");
    return online(c, mode, L, B, n, out_dev);
}

ct_status ct_mac_check_device(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                              ct_check_result *out_dev) {
    if (!c) return CT_EINVAL;
    if (mode != CT_MODE_SPDZ2K && mode != CT_MODE_COMPACT) return fail(c, CT_EINVAL, "unknown mode");
    const bool compact = mode == CT_MODE_COMPACT;
    ct_status s = validate(c, L, B, n, NEED_INPUTS | NEED_TRIPLE | NEED_OUT | (compact ? NEED_CVEC : 0));
    if (s != CT_OK) return s;
    if (!aligned16(out_dev)) return fail(c, CT_EINVAL, "out_dev is null or misaligned");
    HIPCHK(c, hipSetDevice(c->device));
    if ((s = stage_layers(c, L, B, n)) != CT_OK) return s;
    if ((s = upload(c, n, 0)) != CT_OK) return s;
    const Sizes sz = max_sizes(L, n);
    LAUNCH(c, ST_ZERO_ACC, launch_zero_acc(c->layers_dev, n, 2, 0, c->stream));
    const int mask = compact ? 0x3 : 0x7;
    LAUNCH(c, ST_CHECK_BATCH, launch_check_batch(c->layers_dev, n, mask, std::max({sz.mk, sz.kn, sz.mn}), c->stream));
    if (compact) LAUNCH(c, ST_CHECK_COMPACT, launch_check_compact(c->layers_dev, n, c->stream));
    LAUNCH(c, ST_FINALIZE, launch_finalize(c->layers_dev, n, out_dev, c->stream));
    return CT_OK;
}

ct_status ct_mac_check(ct_ctx *c, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                       ct_check_result *out) {
    if (!c) return CT_EINVAL;
    if (!out) return fail(c, CT_EINVAL, "null result array");
    ct_status s = ct_mac_check_device(c, mode, L, B, n, c->res_dev);
    if (s != CT_OK) return s;
    HIPCHK(c, hipMemcpyAsync(c->res_host, c->res_dev, sizeof(ct_check_result) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool ok = true;
    for (int l = 0; l < n; l++) {
        out[l] = c->res_host[l];
        ok = ok && c->res_host[l].accept;
    }
    return ok ? CT_OK : CT_ABORT;
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
    if (t->group_m < 1 || t->split_target < 0 || t->split_target > MAX_STEPS_PER_SPLIT)
        return fail(c, CT_EINVAL, "invalid tuning");
    c->fallback = GemmTuning{t->group_m, t->xcd_remap ? 1 : 0, t->split_target};
    c->tuned.clear();
    return CT_OK;
}

ct_status ct_get_tuning(const ct_ctx *c, ct_mode mode, const ct_layer_desc *L, int n, ct_tuning *out) {
    if (!c || !L || !out || n < 1) return CT_EINVAL;
    const GemmTuning t = tuning_for(c, shape_class(mode, L, n));
    out->group_m = t.group_m;
    out->xcd_remap = t.xcd_remap;
    out->split_target = t.split_target;
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
    const double saved_ms = c->stage_ms[ST_RING_GEMM];
    const int64_t saved_n = c->stage_n[ST_RING_GEMM];
    static const int groups[] = {1, 2, 4, 8, 16, 64};
    static const int splits[] = {0, 16, 32, 64, 128};
    GemmTuning best = c->fallback;
    double best_ms = 1e30;
    for (int xcd = 0; xcd < 2; xcd++)
        for (int g : groups)
            for (int sp : splits) {
                c->forcing = true;
                c->forced = GemmTuning{g, xcd, sp};
                s = online(c, mode, L, B, n, nullptr);  // warm-up
                if (s == CT_OK) {
                    HIPCHK(c, fold_timing(c));
                    c->stage_ms[ST_RING_GEMM] = 0;
                    c->stage_n[ST_RING_GEMM] = 0;
                    for (int r = 0; r < reps && s == CT_OK; r++) s = online(c, mode, L, B, n, nullptr);
                }
                if (s == CT_OK) {
                    HIPCHK(c, fold_timing(c));
                    const double ms = c->stage_ms[ST_RING_GEMM] / reps;
                    if (c->stage_n[ST_RING_GEMM] > 0 && ms < best_ms) {
                        best_ms = ms;
                        best = c->forced;
                    }
                }
                c->forcing = false;
                if (s != CT_OK) return s;
            }
    c->stage_ms[ST_RING_GEMM] = saved_ms;
    c->stage_n[ST_RING_GEMM] = saved_n;
    if (!was_timing) {
        c->timing = false;
    }
    c->tuned[shape_class(mode, L, n)] = best;
    if (best_out) {
        best_out->group_m = best.group_m;
        best_out->xcd_remap = best.xcd_remap;
        best_out->split_target = best.split_target;
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
