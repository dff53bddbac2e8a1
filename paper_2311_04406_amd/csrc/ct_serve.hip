// ct_serve.hip -- the request server of the C ABI (ct_server_*).
//
// A worker thread owns the context while the server lives.  It takes
// submitted requests in order of their scheduled arrival, forms batches with
// the policy of ct_sched.h whenever one of its slots is free, and runs each
// batch on that slot's stream: the dealer for the TAG and PREP requests of
// the batch (not for a TAG whose layer a PREP has dealt already), the online
// phase for its TAG requests, then the MAC checks of its CHECK requests, then
// a copy of the check results to pinned host memory and an event.  Slots run
// concurrently, so batches admitted while others are on the device overlap
// with them.  Completions carry the scheduled arrival, admission and
// completion times on one host clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "compacttag.h"
#include "ct_host.h"
#include "ct_sched.h"

using namespace ct;

namespace {

constexpr int MAX_SLOTS = 8;
constexpr int MAX_BATCH = 256;

struct Slot {
    hipStream_t stream = nullptr;
    Lane deal, online, check;  // one lane per phase: a phase never waits for the upload of another
    hipEvent_t done = nullptr;
    bool busy = false;
    bool failed = false;
    std::string error;
    Batch batch;
    std::vector<int> check_items;  // batch.items index of each executed CHECK, in launch order
};

}  // namespace

struct ct_server {
    ct_ctx *ctx = nullptr;
    ct_server_params p{};
    char *base = nullptr;
    Scheduler sched;
    std::vector<Slot> slots;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_in, cv_done;
    std::vector<PendingReq> inbox;
    std::deque<ct_completion> outbox;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    std::string err;
    std::chrono::steady_clock::time_point epoch;

    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - epoch).count();
    }
};

namespace {

ct_layer_bufs layer_bufs(char *base, const Resident &r) {
    const LayerLayout o = layer_layout(r.layer.M, r.layer.K, r.layer.N);
    char *b = base + r.off;
    auto at = [&](size_t off) { return reinterpret_cast<ct_u128 *>(b + off); };
    ct_layer_bufs B;
    std::memset(&B, 0, sizeof(B));
    ct_u128 **mk[4][2] = {{&B.X[0], &B.X[1]}, {&B.tX[0], &B.tX[1]}, {&B.A[0], &B.A[1]}, {&B.tA[0], &B.tA[1]}};
    ct_u128 **kn[4][2] = {{&B.Y[0], &B.Y[1]}, {&B.tY[0], &B.tY[1]}, {&B.B[0], &B.B[1]}, {&B.tB[0], &B.tB[1]}};
    ct_u128 **mn[6][2] = {{&B.C[0], &B.C[1]}, {&B.tC[0], &B.tC[1]}, {&B.R[0], &B.R[1]},
                          {&B.tR[0], &B.tR[1]}, {&B.Z[0], &B.Z[1]}, {&B.tZ[0], &B.tZ[1]}};
    for (int i = 0; i < 4; i++)
        for (int q = 0; q < 2; q++) {
            *mk[i][q] = at(o.mk[2 * i + q]);
            *kn[i][q] = at(o.kn[2 * i + q]);
        }
    for (int i = 0; i < 6; i++)
        for (int q = 0; q < 2; q++) *mn[i][q] = at(o.mn[2 * i + q]);
    B.E = at(o.E);
    B.U = at(o.U);
    B.D = at(o.D);
    B.cvec = at(o.cvec);
    B.work = r.work_bytes ? reinterpret_cast<ct_u128 *>(base + r.work_off) : nullptr;
    return B;
}

// Enqueues a batch on its slot.  Runs on the worker thread, outside the lock;
// the layer lists were read from the scheduler under the lock: dealL/dealB
// the layers the dealer writes (TAG and PREP), onL/onB those whose online
// phase runs (TAG), chkL/chkB those checked (CHECK).
void launch_batch(ct_server *s, Slot &sl, std::vector<ct_layer_desc> &dealL, std::vector<ct_layer_bufs> &dealB,
                  std::vector<ct_layer_desc> &onL, std::vector<ct_layer_bufs> &onB,
                  std::vector<ct_layer_desc> &chkL, std::vector<ct_layer_bufs> &chkB) {
    ct_ctx *c = s->ctx;
    const ct_mode mode = (ct_mode)s->p.mode;
    sl.failed = false;
    sl.error.clear();
    ct_status st = CT_OK;
    const int nd = (int)dealL.size(), nt = (int)onL.size(), nc = (int)chkL.size();
    if (nd > 0) st = run_deal(c, sl.deal, dealL.data(), dealB.data(), nd, 1);
    if (st == CT_OK && nt > 0) st = run_online(c, sl.online, mode, onL.data(), onB.data(), nt, nullptr);
    if (st == CT_OK && nc > 0) {
        st = run_check(c, sl.check, mode, chkL.data(), chkB.data(), nc, sl.check.res_dev);
        if (st == CT_OK &&
            hipMemcpyAsync(sl.check.res_host, sl.check.res_dev, sizeof(ct_check_result) * nc, hipMemcpyDeviceToHost,
                           sl.stream) != hipSuccess)
            st = fail(c, CT_EDEVICE, "result copy failed");
    }
    if (st != CT_OK) {
        sl.failed = true;
        sl.error = c->err;
    }
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) {
        // nothing to wait for: complete the batch at the next poll
        sl.failed = true;
        if (sl.error.empty()) sl.error = "hipEventRecord failed";
        (void)hipStreamSynchronize(sl.stream);
    }
    sl.busy = true;
}

// The batch on sl has completed (or failed): completions, then the policy.
void finish_batch(ct_server *s, Slot &sl, bool device_ok, double now) {
    std::lock_guard<std::mutex> lk(s->mu);
    const bool ok = device_ok && !sl.failed;
    if (!ok) s->err = sl.error.empty() ? "device error" : sl.error;
    std::vector<int> check_pos(sl.batch.items.size(), -1);
    for (size_t j = 0; j < sl.check_items.size(); j++) check_pos[sl.check_items[j]] = (int)j;
    for (size_t i = 0; i < sl.batch.items.size(); i++) {
        const BatchItem &it = sl.batch.items[i];
        ct_completion cp;
        std::memset(&cp, 0, sizeof(cp));
        cp.id = it.req_id;
        cp.kind = it.kind;
        cp.layer = it.resident;
        cp.arrival_us = it.arrival_us;
        cp.admit_us = sl.batch.admit_us;
        cp.done_us = now;
        cp.batch_size = (int32_t)sl.batch.items.size();
        cp.slot = sl.batch.slot;
        if (it.status != CT_OK) {
            cp.status = it.status;
        } else if (!ok) {
            cp.status = CT_EDEVICE;
        } else if (it.kind == REQ_CHECK) {
            cp.result = sl.check.res_host[check_pos[i]];
            cp.status = cp.result.accept ? CT_OK : CT_ABORT;
        } else {
            cp.status = CT_OK;
        }
        s->outbox.push_back(cp);
    }
    s->completed += (int64_t)sl.batch.items.size();
    s->sched.finish(sl.batch, ok);
    sl.busy = false;
    s->cv_done.notify_all();
}

void worker_main(ct_server *s) {
    (void)hipSetDevice(s->ctx->device);
    std::vector<ct_layer_desc> dealL, onL, chkL;
    std::vector<ct_layer_bufs> dealB, onB, chkB;
    while (true) {
        bool stopping;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (const PendingReq &r : s->inbox) s->sched.submit(r);
            s->inbox.clear();
            stopping = s->stop;
        }
        bool progressed = false;
        int busy = 0;
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) {
                busy++;
                continue;
            }
            finish_batch(s, sl, q == hipSuccess, s->now_us());
            progressed = true;
        }
        if (stopping) {
            if (busy == 0) break;
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            continue;
        }
        while (true) {
            Batch b;
            dealL.clear(); dealB.clear(); onL.clear(); onB.clear(); chkL.clear(); chkB.clear();
            Slot *sl = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (!s->sched.next_batch(s->now_us(), b)) break;
                sl = &s->slots[b.slot];
                sl->check_items.clear();
                for (size_t i = 0; i < b.items.size(); i++) {
                    const BatchItem &it = b.items[i];
                    if (it.status != CT_OK) continue;
                    const Resident *r = s->sched.resident(it.resident);
                    if (it.kind == REQ_TAG || it.kind == REQ_PREP) {
                        if (!it.online_only) {
                            dealL.push_back(r->layer);
                            dealB.push_back(layer_bufs(s->base, *r));
                        }
                        if (it.kind == REQ_TAG) {
                            onL.push_back(r->layer);
                            onB.push_back(layer_bufs(s->base, *r));
                        }
                    } else {
                        chkL.push_back(r->layer);
                        chkB.push_back(layer_bufs(s->base, *r));
                        sl->check_items.push_back((int)i);
                    }
                }
                sl->batch = b;
            }
            launch_batch(s, *sl, dealL, dealB, onL, onB, chkL, chkB);
            progressed = true;
            busy++;
        }
        if (progressed) continue;
        if (busy > 0) {
            std::this_thread::sleep_for(std::chrono::microseconds(10));
        } else {
            // idle: sleep until a submission, the next scheduled arrival or 1 ms
            std::unique_lock<std::mutex> lk(s->mu);
            const double next = s->sched.next_arrival();
            double wait_us = 1000.0;
            if (next >= 0) wait_us = std::min(wait_us, std::max(0.0, next - s->now_us()));
            if (s->inbox.empty() && !s->stop && wait_us > 0)
                s->cv_in.wait_for(lk, std::chrono::microseconds((int64_t)wait_us + 1));
        }
    }
}

ct_status sfail(ct_server *s, ct_status st, const std::string &msg) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->err = msg;
    return st;
}

void free_slots(ct_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        lane_free(sl.deal);
        lane_free(sl.online);
        lane_free(sl.check);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    s->slots.clear();
}

}  // namespace

extern "C" {

ct_status ct_server_create(ct_ctx *ctx, const ct_server_params *p, ct_server **out) {
    if (!ctx || !p || !out) return CT_EINVAL;
    *out = nullptr;
    if (!p->arena || (reinterpret_cast<uintptr_t>(p->arena) % ARENA_ALIGN) != 0)
        return fail(ctx, CT_EINVAL, "arena is null or not 256-byte aligned");
    if (p->arena_bytes < ARENA_ALIGN) return fail(ctx, CT_EINVAL, "arena is too small");
    if (p->slots < 1 || p->slots > MAX_SLOTS) return fail(ctx, CT_EINVAL, "slots must be in [1, 8]");
    if (p->max_batch < 1 || p->max_batch > MAX_BATCH) return fail(ctx, CT_EINVAL, "max_batch must be in [1, 256]");
    if (p->mode != CT_MODE_SPDZ2K && p->mode != CT_MODE_COMPACT) return fail(ctx, CT_EINVAL, "unknown mode");
    if (ctx->eb != 16) return fail(ctx, CT_EINVAL, "the server runs the k = s = 64 parameter set");
    if (ctx->np != 2) return fail(ctx, CT_EINVAL, "the server runs two parties");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CT_EDEVICE, "hipSetDevice failed");
    ct_server *s = new ct_server();
    s->ctx = ctx;
    s->p = *p;
    s->base = static_cast<char *>(p->arena);
    s->sched.reset(p->arena_bytes, p->slots, p->max_batch);
    s->slots.resize(p->slots);
    for (Slot &sl : s->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = lane_init(sl.deal, sl.stream, p->max_batch);
        if (e == hipSuccess) e = lane_init(sl.online, sl.stream, p->max_batch);
        if (e == hipSuccess) e = lane_init(sl.check, sl.stream, p->max_batch);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            free_slots(s);
            delete s;
            return fail(ctx, CT_EDEVICE, std::string("ct_server_create: ") + hipGetErrorString(e));
        }
    }
    s->epoch = std::chrono::steady_clock::now();
    s->worker = std::thread(worker_main, s);
    *out = s;
    return CT_OK;
}

double ct_server_now_us(const ct_server *s) { return s ? s->now_us() : 0.0; }

ct_status ct_server_submit(ct_server *s, const ct_request *r, int n) {
    if (!s || (n > 0 && !r) || n < 0) return CT_EINVAL;
    for (int i = 0; i < n; i++) {
        const ct_layer_desc &d = r[i].layer;
        if (r[i].kind != CT_REQ_TAG && r[i].kind != CT_REQ_CHECK && r[i].kind != CT_REQ_PREP)
            return sfail(s, CT_EINVAL, "request " + std::to_string(i) + ": unknown kind");
        if (d.M < 1 || d.K < 1 || d.N < 1 || d.M >= (1LL << 31) || d.K >= (1LL << 21) || d.N >= (1LL << 22) ||
            d.f != 0 || d.in_bits < 0 || d.in_bits > 63 || d.layer_id >= (1ULL << 48) || d.compress < 0 ||
            d.compress > CT_COMPRESS_AUTO || d.reserved != 0 || d.conv_c != 0)
            return sfail(s, CT_EINVAL, "request " + std::to_string(i) + ": invalid layer");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (int i = 0; i < n; i++) s->inbox.push_back(PendingReq{r[i].id, r[i].kind, r[i].layer, r[i].arrival_us});
        s->submitted += n;
    }
    s->cv_in.notify_one();
    return CT_OK;
}

ct_status ct_server_poll(ct_server *s, ct_completion *out, int max, int *count) {
    if (!s || !count || (max > 0 && !out)) return CT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int k = 0;
    while (k < max && !s->outbox.empty()) {
        out[k++] = s->outbox.front();
        s->outbox.pop_front();
    }
    *count = k;
    return CT_OK;
}

ct_status ct_server_drain(ct_server *s, double timeout_s) {
    if (!s) return CT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool done = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                          [&] { return s->completed >= s->submitted; });
    if (!done) {
        s->err = "drain timed out with " + std::to_string(s->submitted - s->completed) + " requests open";
        return CT_EDEVICE;
    }
    return CT_OK;
}

ct_status ct_server_layer(ct_server *s, int64_t id, ct_layer_desc *desc, ct_layer_bufs *bufs) {
    if (!s || !desc || !bufs) return CT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const Resident *r = s->sched.resident(id);
    if (!r || !r->ready) {
        s->err = "layer " + std::to_string(id) + " is not resident";
        return CT_EINVAL;
    }
    *desc = r->layer;
    *bufs = layer_bufs(s->base, *r);
    bufs->work = nullptr;
    return CT_OK;
}

ct_status ct_server_stats(ct_server *s, ct_server_counts *out) {
    if (!s || !out) return CT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const SchedStats &st = s->sched.stats();
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = st.rejected;
    out->converted = st.converted;
    out->evictions = st.evictions;
    out->batches = st.batches;
    out->max_batch = st.max_batch;
    out->arena_bytes = s->sched.arena().size();
    out->arena_peak = st.arena_peak;
    out->arena_used = s->sched.arena().used();
    out->resident_layers = (int64_t)s->sched.residents().size();
    out->duplicates = st.duplicates;
    out->prepared = st.prepared;
    out->online_only = st.online_only;
    return CT_OK;
}

ct_status ct_server_destroy(ct_server *s) {
    if (!s) return CT_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_in.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    free_slots(s);
    delete s;
    return CT_OK;
}

const char *ct_server_last_error(ct_server *s) {
    if (!s) return "null server";
    std::lock_guard<std::mutex> lk(s->mu);
    return s->err.c_str();
}

}  // extern "C"
