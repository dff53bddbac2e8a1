// ct_sched.h -- admission, batching and residency policy of the request
// server (ct_serve.hip).  Plain C++ with no HIP calls, so the policy runs and
// is tested on the host alone; the server glues it to streams and kernels.
//
// Requests are tag generation (TAG: the dealer draws the layer's inputs and
// triple into freshly admitted memory, then the online phase computes its
// outputs and tags), verification (CHECK: the MAC checks of a resident
// layer of the requested shape whose tags are complete; with none resident
// it runs as a TAG) and preprocessing (PREP: only the dealer, ahead of the
// TAG request of the same layer -- the offline phase; that TAG then runs
// only the online phase on the prepared layer).  Admission is by footprint in one device arena: a TAG
// needs the layer's resident bytes plus its transient workspace; completed
// layers stay resident (shares, tags, public values) for later CHECKs and
// are evicted least recently used first when a TAG does not fit.  Batches
// are formed continuously: whenever a slot (stream) is free, every request
// that has arrived and fits goes into the next batch, in arrival order,
// up to the batch limit; a request that does not fit holds back the ones
// behind it (no overtaking), so admission stays first come, first served.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "compacttag.h"

namespace ct {

constexpr size_t ARENA_ALIGN = 256;

inline size_t arena_round(size_t bytes) { return (bytes + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN; }

// Byte offsets of one layer's arrays inside its resident allocation, in
// this order, each ARENA_ALIGN-aligned: X, tX, A, tA of both parties (M x K);
// Y, tY, B, tB (K x N); C, tC, R, tR, Z, tZ (M x N); E; U; D; cvec.
struct LayerLayout {
    size_t mk[8], kn[8], mn[12], E, U, D, cvec, total;
};

inline LayerLayout layer_layout(int64_t M, int64_t K, int64_t N) {
    LayerLayout o;
    const size_t el = sizeof(ct_u128);
    const size_t bmk = arena_round((size_t)(M * K) * el), bkn = arena_round((size_t)(K * N) * el),
                 bmn = arena_round((size_t)(M * N) * el);
    size_t off = 0;
    for (int i = 0; i < 8; i++, off += bmk) o.mk[i] = off;
    for (int i = 0; i < 8; i++, off += bkn) o.kn[i] = off;
    for (int i = 0; i < 12; i++, off += bmn) o.mn[i] = off;
    o.E = off; off += bmk;
    o.U = off; off += bkn;
    o.D = off; off += bmn;
    // compact vectors for either compressed dimension
    o.cvec = off; off += arena_round((size_t)(3 * K + 10 * (M > N ? M : N)) * el);
    o.total = off;
    return o;
}

inline size_t layer_work_bytes(int64_t M, int64_t K, int64_t N) {
    return arena_round((size_t)CT_WORK_LEN(M, K, N) * sizeof(ct_u128));
}

// First-fit allocator over the offsets [0, size) of one arena.  Blocks are
// multiples of ARENA_ALIGN; freed neighbours coalesce.
class Arena {
   public:
    static constexpr size_t NONE = SIZE_MAX;

    explicit Arena(size_t size = 0) { reset(size); }

    void reset(size_t size) {
        size_ = size / ARENA_ALIGN * ARENA_ALIGN;
        used_ = 0;
        free_.clear();
        if (size_) free_[0] = size_;
    }

    size_t alloc(size_t bytes) {
        bytes = arena_round(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            return off;
        }
        return NONE;
    }

    void release(size_t off, size_t bytes) {
        bytes = arena_round(std::max<size_t>(bytes, 1));
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
    const std::map<size_t, size_t> &free_map() const { return free_; }

   private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

enum ReqKind : int32_t { REQ_TAG = 0, REQ_CHECK = 1, REQ_PREP = 2 };

struct PendingReq {
    int64_t id;
    int32_t kind;
    ct_layer_desc layer;
    double arrival_us;
};

// A layer whose buffers live in the arena.
struct Resident {
    int64_t id = 0;  // id of the TAG request that produced it
    ct_layer_desc layer{};
    size_t off = 0, bytes = 0;       // resident allocation
    size_t work_off = 0, work_bytes = 0;  // workspace, held while its TAG is in flight
    int pins = 0;                    // batches in flight that use it
    bool ready = false;              // its tags are complete
    bool prepared = false;           // written by a PREP: dealt for a later TAG, online phase not run
    bool dealt = false;              // (prepared) the dealer has completed
    uint64_t last_use = 0;
};

struct BatchItem {
    int64_t req_id = 0;
    int32_t requested = REQ_TAG;  // kind as submitted
    int32_t kind = REQ_TAG;       // kind as executed
    int32_t status = CT_OK;       // CT_ENOMEM: larger than the arena; CT_EINVAL: the id of a resident
                                  // layer (neither is executed)
    int64_t resident = -1;        // id of the resident layer it writes (TAG, PREP) or verifies (CHECK)
    int32_t online_only = 0;      // a TAG on a prepared layer: the online phase only
    double arrival_us = 0;
};

struct Batch {
    int slot = -1;
    double admit_us = 0;
    std::vector<BatchItem> items;
};

struct SchedStats {
    int64_t submitted = 0, admitted = 0, finished = 0, rejected = 0, converted = 0, evictions = 0, batches = 0;
    int64_t duplicates = 0;  // requests refused because their id named a resident layer
    int64_t prepared = 0;    // PREP requests admitted
    int64_t online_only = 0; // TAG requests that found their layer prepared
    int64_t max_batch = 0;
    size_t arena_peak = 0;
};

class Scheduler {
   public:
    Scheduler() = default;
    Scheduler(size_t arena_bytes, int slots, int max_batch) { reset(arena_bytes, slots, max_batch); }

    void reset(size_t arena_bytes, int slots, int max_batch) {
        arena_.reset(arena_bytes);
        slot_busy_.assign(std::max(slots, 1), false);
        max_batch_ = std::max(max_batch, 1);
        queue_.clear();
        residents_.clear();
        stats_ = SchedStats();
        clock_ = 0;
    }

    // Requests enter in order of their scheduled arrival (stable for ties).
    void submit(const PendingReq &r) {
        auto it = queue_.end();
        while (it != queue_.begin() && std::prev(it)->arrival_us > r.arrival_us) --it;
        queue_.insert(it, r);
        stats_.submitted++;
    }

    int free_slot() const {
        for (size_t i = 0; i < slot_busy_.size(); i++)
            if (!slot_busy_[i]) return (int)i;
        return -1;
    }
    int busy_slots() const { return (int)std::count(slot_busy_.begin(), slot_busy_.end(), true); }
    size_t queued() const { return queue_.size(); }
    double next_arrival() const { return queue_.empty() ? -1.0 : queue_.front().arrival_us; }

    // Forms the next batch from the requests that have arrived by now_us, for
    // a free slot.  Returns false (and forms nothing) if no slot is free or
    // no arrived request can be admitted.  Requests larger than the whole
    // arena are returned in the batch with status CT_ENOMEM, requests whose id
    // is that of a resident layer with CT_EINVAL; neither is executed.
    bool next_batch(double now_us, Batch &b) {
        const int slot = free_slot();
        b = Batch();
        if (slot < 0) return false;
        while (!queue_.empty() && (int)b.items.size() < max_batch_) {
            const PendingReq &r = queue_.front();
            if (r.arrival_us > now_us) break;
            BatchItem it;
            it.req_id = r.id;
            it.requested = it.kind = r.kind;
            it.arrival_us = r.arrival_us;
            if (residents_.count(r.id)) {
                // the id of a layer still resident (maybe in flight): refused,
                // so that layer and its workspace are never taken over
                it.status = CT_EINVAL;
                b.items.push_back(it);
                queue_.pop_front();
                stats_.duplicates++;
                continue;
            }
            if (r.kind == REQ_CHECK) {
                Resident *t = newest_ready(r.layer);
                if (t) {
                    t->pins++;
                    t->last_use = ++clock_;
                    it.resident = t->id;
                    b.items.push_back(it);
                    queue_.pop_front();
                    continue;
                }
                it.kind = REQ_TAG;  // nothing of this shape to verify: run it as a TAG
            }
            if (r.kind == REQ_TAG) {
                Resident *pr = prepared_for(r.layer);
                if (pr) {
                    if (!pr->dealt) break;  // its preparation is still in flight; nothing overtakes
                    // the online phase needs the workspace again; the
                    // prepared layer is pinned so that no eviction takes it
                    const size_t work = layer_work_bytes(r.layer.M, r.layer.K, r.layer.N);
                    pr->pins++;
                    size_t woff = work ? Arena::NONE : 0;
                    while (work && (woff = arena_.alloc(work)) == Arena::NONE)
                        if (!evict_one()) break;
                    pr->pins--;
                    if (woff == Arena::NONE) break;  // waits for memory
                    Resident res = *pr;
                    residents_.erase(pr->id);
                    res.id = r.id;
                    res.prepared = false;
                    res.work_off = woff;
                    res.work_bytes = work;
                    res.pins = 1;
                    res.last_use = ++clock_;
                    residents_[r.id] = res;
                    it.resident = r.id;
                    it.online_only = 1;
                    stats_.online_only++;
                    b.items.push_back(it);
                    queue_.pop_front();
                    continue;
                }
            }
            const LayerLayout lay = layer_layout(r.layer.M, r.layer.K, r.layer.N);
            const size_t work = layer_work_bytes(r.layer.M, r.layer.K, r.layer.N);
            if (lay.total + work > arena_.size()) {
                it.status = CT_ENOMEM;
                b.items.push_back(it);
                queue_.pop_front();
                stats_.rejected++;
                continue;
            }
            size_t off = Arena::NONE, woff = Arena::NONE;
            while (true) {
                off = arena_.alloc(lay.total);
                if (off != Arena::NONE) {
                    woff = work ? arena_.alloc(work) : 0;
                    if (woff != Arena::NONE) break;
                    arena_.release(off, lay.total);
                    off = Arena::NONE;
                }
                if (!evict_one()) break;
            }
            if (off == Arena::NONE) break;  // waits for memory; nothing overtakes it
            Resident res;
            res.id = r.id;
            res.layer = r.layer;
            res.off = off;
            res.bytes = lay.total;
            res.work_off = woff;
            res.work_bytes = work;
            res.pins = 1;
            res.last_use = ++clock_;
            res.prepared = r.kind == REQ_PREP;
            residents_[r.id] = res;
            if (it.kind != it.requested) stats_.converted++;
            if (r.kind == REQ_PREP) stats_.prepared++;
            it.resident = r.id;
            b.items.push_back(it);
            queue_.pop_front();
        }
        if (b.items.empty()) return false;
        b.slot = slot;
        b.admit_us = now_us;
        slot_busy_[slot] = true;
        stats_.batches++;
        stats_.admitted += (int64_t)b.items.size();
        stats_.max_batch = std::max<int64_t>(stats_.max_batch, (int64_t)b.items.size());
        stats_.arena_peak = std::max(stats_.arena_peak, arena_.used());
        return true;
    }

    // The batch has completed on the device: TAG layers become ready (their
    // workspace is released), PREP layers dealt (likewise), CHECK pins are
    // dropped, the slot is free.  A TAG or PREP that failed (ok == false)
    // releases its layer.
    void finish(const Batch &b, bool ok = true) {
        for (const BatchItem &it : b.items) {
            stats_.finished++;
            if (it.status != CT_OK) continue;
            auto r = residents_.find(it.resident);
            if (r == residents_.end()) continue;
            Resident &res = r->second;
            res.pins--;
            res.last_use = ++clock_;
            if (it.kind == REQ_TAG || it.kind == REQ_PREP) {
                if (res.work_bytes) arena_.release(res.work_off, res.work_bytes);
                res.work_bytes = 0;
                if (ok) {
                    if (it.kind == REQ_TAG) res.ready = true;
                    else res.dealt = true;
                } else {
                    arena_.release(res.off, res.bytes);
                    residents_.erase(r);
                }
            }
        }
        if (b.slot >= 0 && b.slot < (int)slot_busy_.size()) slot_busy_[b.slot] = false;
    }

    const Resident *resident(int64_t id) const {
        auto it = residents_.find(id);
        return it == residents_.end() ? nullptr : &it->second;
    }
    const std::unordered_map<int64_t, Resident> &residents() const { return residents_; }
    const Arena &arena() const { return arena_; }
    const SchedStats &stats() const { return stats_; }

   private:
    // Most recently produced ready layer of the same shape (M, K, N).
    Resident *newest_ready(const ct_layer_desc &d) {
        Resident *best = nullptr;
        for (auto &kv : residents_) {
            Resident &r = kv.second;
            if (!r.ready || r.layer.M != d.M || r.layer.K != d.K || r.layer.N != d.N) continue;
            if (!best || r.id > best->id) best = &r;
        }
        return best;
    }

    // The dealt or in-flight prepared layer of a TAG's layer (same shape,
    // seed and layer id), if any.
    Resident *prepared_for(const ct_layer_desc &d) {
        for (auto &kv : residents_) {
            Resident &r = kv.second;
            if (r.prepared && r.layer.M == d.M && r.layer.K == d.K && r.layer.N == d.N && r.layer.seed == d.seed &&
                r.layer.layer_id == d.layer_id)
                return &r;
        }
        return nullptr;
    }

    // Evicts the least recently used complete layer that no batch in flight
    // uses -- a ready one if there is any, else a dealt prepared one (whose
    // TAG then deals its layer again); false if there is none.
    bool evict_one() {
        auto victim = residents_.end();
        for (int pass = 0; pass < 2 && victim == residents_.end(); pass++)
            for (auto it = residents_.begin(); it != residents_.end(); ++it) {
                const Resident &r = it->second;
                const bool done = pass == 0 ? r.ready : (r.prepared && r.dealt);
                if (!done || r.pins > 0) continue;
                if (victim == residents_.end() || r.last_use < victim->second.last_use) victim = it;
            }
        if (victim == residents_.end()) return false;
        arena_.release(victim->second.off, victim->second.bytes);
        residents_.erase(victim);
        stats_.evictions++;
        return true;
    }

    Arena arena_;
    std::vector<bool> slot_busy_;
    int max_batch_ = 1;
    std::deque<PendingReq> queue_;
    std::unordered_map<int64_t, Resident> residents_;
    SchedStats stats_;
    uint64_t clock_ = 0;
};

}  // namespace ct
