// ct_host.h -- host-side internals shared by the C ABI (ct_api.hip), the
// captured plans and the request server (ct_serve.hip).
//
// A Lane is everything one in-order execution of the path needs besides the
// layer buffers: a HIP stream, device-resident tables (one LayerDev record
// per layer, the matrix-core problem and packing-job lists), their pinned
// host staging copies, the per-layer check accumulators and a result array.
// The context owns one lane for its plain calls; a captured plan and every
// slot of a server own one each, so their work can be in flight together.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <unordered_map>
#include <vector>

#include "compacttag.h"
#include "ct_internal.h"

namespace ct {

struct Lane {
    hipStream_t stream = nullptr;
    int max_layers = 0, max_probs = 0, max_jobs = 0;
    LayerDev *layers_dev = nullptr, *layers_host = nullptr;
    GemmProb *gemm_dev = nullptr, *gemm_host = nullptr;
    PackJob *pack_dev = nullptr, *pack_host = nullptr;
    SkinnyProb *skinny_dev = nullptr, *skinny_host = nullptr;
    u128 *acc_dev = nullptr;
    ct_check_result *res_dev = nullptr, *res_host = nullptr;
    uint32_t *sync_dev = nullptr;      // counters of the persistent launch (64 bytes)
    hipEvent_t upload_done = nullptr;  // the staging copies may be rewritten once this has completed
    bool timed = false;                // per-launch event timing (the context's own lane only)
};

// Allocates the lane's tables for up to max_layers layers (the stream is the
// caller's).  On failure the lane is left for lane_free.
hipError_t lane_init(Lane &ln, hipStream_t stream, int max_layers);
void lane_free(Lane &ln);

}  // namespace ct

// Kernel stages, for the optional per-launch timing (ct_set_timing).
enum Stage : int {
    ST_DEAL_LIFT, ST_FILL_ZERO, ST_DEAL_AUTH, ST_DEAL_SKINNY, ST_ZERO_ACC, ST_OPEN_U, ST_ROW_PASS, ST_PACK,
    ST_COPY_BASE, ST_RING_GEMM, ST_POST, ST_COMPACT_FINAL, ST_CHECK_BATCH, ST_CHECK_COMPACT, ST_FINALIZE,
    ST_COL_TAG, ST_CONV_COMPRESS, ST_NP_OPEN, ST_NP_SKINNY, ST_NP_COMPRESS, ST_NP_GEMV, ST_OPEN_PACK, ST_PERSIST,
    ST_COUNT
};

struct ct_ctx {
    int device = 0;
    int eb = 16;  // bytes per ring element: 16 (k = s = 64, Z_{2^128}) or 8 (k = s = 32, Z_{2^64})
    int np = 2;   // parties simulated
    uint64_t delta[CT_MAX_PARTIES] = {};  // key shares [Delta]_p, p < np
    int num_cus = 256;
    ct::Lane main;
    // second lane for the matrix-core layers of a mixed online call, and the
    // events that fork it from and join it to the main stream
    ct::Lane side;
    hipEvent_t fork = nullptr, join = nullptr;
    bool overlap = true;  // mixed batches on two streams (ct_set_overlap)
    int launch_mode = CT_LAUNCH_STAGED;  // ct_set_launch
    uint64_t launch_wait = CT_LAUNCH_WAIT_DEFAULT;  // ct_set_launch_wait
    std::string err;
    // per-launch timing: event pairs recorded around each kernel of the main lane
    bool timing = false;
    std::vector<hipEvent_t> ev_start, ev_end;
    std::vector<int> ev_stage;
    int ev_used = 0;
    double stage_ms[ST_COUNT] = {};
    int64_t stage_n[ST_COUNT] = {};
    // launch configuration of the matrix-core products per shape class
    std::unordered_map<uint64_t, ct::GemmTuning> tuned;
    ct::GemmTuning fallback = {1, 0, 0, CT_TILE_AUTO};
    bool forcing = false;
    ct::GemmTuning forced = {1, 0, 0, CT_TILE_AUTO};
    // ct_tag_linear_check_static: this device's static workspace (its device
    // address, from hipGetSymbolAddress at ct_create) and the host copy of a
    // call's buffer records with their workspace pointers redirected into it
    // (max_layers records, allocated at ct_create)
    void *static_work = nullptr;
    std::vector<ct_layer_bufs> static_bufs;
};

namespace ct {

// The phases of the path on a lane.  Each validates, stages and uploads its
// tables on ln.stream, then enqueues its kernels there; nothing blocks except
// the wait for the lane's previous upload.
ct_status run_deal(ct_ctx *c, Lane &ln, const ct_layer_desc *L, const ct_layer_bufs *B, int n, int with_inputs);
ct_status run_online(ct_ctx *c, Lane &ln, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                     ct_check_result *out_dev);
ct_status run_check(ct_ctx *c, Lane &ln, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                    ct_check_result *out_dev);

// Online phase split in two for capture: prepare validates and uploads the
// tables (outside a capture), enqueue only launches kernels.
struct OnlineLaunch {
    int n = 0, nm = 0, njobs = 0, pack_tiles = 0, total_tiles = 0, variants = 0, flags = 0, zero_what = 0;
    int open_tiles = 0;       // k_open_pack tiles of the largest fused layer
    bool any_open_u = false;  // a layer that k_open_u opens (not fused)
    bool any_accum = false, compact = false, check = false, any_cm = false, any_conv_n = false;
    ct_mode mode = CT_MODE_COMPACT;
    GemmTuning tu;
    int64_t max_zero = 0, max_kn_items = 0, max_row_items = 0, max_mn = 0, max_mn_items = 0, max_col_tag = 0,
            max_conv_items = 0;
    // n-party path
    int64_t max_open = 0, max_skinny_items = 0, max_compress_items = 0, max_gemv_items = 0, max_cvec_np = 0;
    bool any_skinny = false, any_unfused = false;  // layers with 2 < N <= SKINNY_MAX_N
    ct_check_result *out_dev = nullptr;
};
ct_status prepare_online(ct_ctx *c, Lane &ln, ct_mode mode, const ct_layer_desc *L, const ct_layer_bufs *B, int n,
                         ct_check_result *out_dev, OnlineLaunch &P, const int *out_index = nullptr);
ct_status enqueue_online(ct_ctx *c, Lane &ln, const OnlineLaunch &P);
// The online phase of a batch that mixes matrix-core layers (N > 8) with
// layers whose products the row pass forms: the matrix-core layers run on
// lane b, forked from lane a's stream, and the others on lane a, joined back
// before anything later on lane a's stream.  The two groups share no data, so
// their kernels overlap (the row pass of a wide classifier is bandwidth-bound,
// the products of convolutions are not).  A batch of one kind runs on lane a.
ct_status prepare_online_split(ct_ctx *c, Lane &a, Lane &b, ct_mode mode, const ct_layer_desc *L,
                               const ct_layer_bufs *B, int n, ct_check_result *out_dev, OnlineLaunch &Pa,
                               OnlineLaunch &Pb, bool &split);
ct_status enqueue_online_split(ct_ctx *c, Lane &a, Lane &b, hipEvent_t fork, hipEvent_t join, const OnlineLaunch &Pa,
                               const OnlineLaunch &Pb, bool split);

ct_status fail(ct_ctx *c, ct_status s, const std::string &msg);

}  // namespace ct
