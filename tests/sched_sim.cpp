// Host-only checks of the request server's policy (ct_sched.h): the arena
// allocator against a granule bitmap, and the scheduler driven by a
// simulated clock (Poisson arrivals, batches that complete after a service
// time proportional to their bytes) with its invariants checked after every
// step.  Prints one "ok ..." line per scenario; exits non-zero on the first
// violated invariant.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "ct_sched.h"

using namespace ct;

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

// ---- arena ----

static void arena_scenario(uint64_t seed) {
    const size_t G = ARENA_ALIGN, n = 2048;
    Arena a(n * G + 100);  // a ragged size rounds down
    CHECK(a.size() == n * G);
    std::vector<int> owner(n, -1);
    std::map<size_t, size_t> live;  // offset -> bytes requested
    std::mt19937_64 rng(seed);
    int id = 0, fails = 0;
    for (int step = 0; step < 20000; step++) {
        if (live.empty() || rng() % 5 < 3) {
            const size_t bytes = 1 + rng() % (G * 40);
            const size_t g = (bytes + G - 1) / G;
            // first-fit reference: lowest maximal free run of at least g granules
            size_t expect = Arena::NONE;
            for (size_t i = 0; i < n;) {
                if (owner[i] != -1) { i++; continue; }
                size_t j = i;
                while (j < n && owner[j] == -1) j++;
                if (j - i >= g) { expect = i * G; break; }
                i = j;
            }
            const size_t off = a.alloc(bytes);
            CHECK(off == expect);
            if (off == Arena::NONE) { fails++; continue; }
            for (size_t k = off / G; k < off / G + g; k++) {
                CHECK(owner[k] == -1);
                owner[k] = id;
            }
            id++;
            live[off] = bytes;
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            const size_t g = (it->second + G - 1) / G;
            for (size_t k = it->first / G; k < it->first / G + g; k++) owner[k] = -1;
            a.release(it->first, it->second);
            live.erase(it);
        }
        size_t used = 0;
        for (auto &kv : live) used += arena_round(kv.second);
        CHECK(a.used() == used);
        // free blocks are exactly the maximal free runs (always coalesced)
        std::map<size_t, size_t> runs;
        for (size_t i = 0; i < n;) {
            if (owner[i] != -1) { i++; continue; }
            size_t j = i;
            while (j < n && owner[j] == -1) j++;
            runs[i * G] = (j - i) * G;
            i = j;
        }
        CHECK(runs == a.free_map());
    }
    for (auto &kv : live) a.release(kv.first, kv.second);
    CHECK(a.used() == 0 && a.free_blocks() == 1 && a.largest_free() == a.size());
    std::printf("ok arena seed=%llu allocs=%d failed_allocs=%d\n", (unsigned long long)seed, id, fails);
}

// ---- scheduler ----

struct Shape { int64_t M, K, N; };

struct InFlight {
    Batch b;
    double end;
};

static size_t footprint(const ct_layer_desc &d) {
    return layer_layout(d.M, d.K, d.N).total + layer_work_bytes(d.M, d.K, d.N);
}

static void sched_scenario(const char *name, uint64_t seed, size_t arena, int slots, int max_batch, int nreq,
                           double rate_per_us, double bytes_per_us, int expect_evictions, int expect_rejects) {
    // shapes: wide (matrix-core path, with workspace) and skinny (N <= 8)
    const std::vector<Shape> shapes = {{64, 576, 300}, {128, 1152, 78}, {70, 100, 130}, {33, 70, 1},
                                       {256, 230, 19}, {40, 2100, 70}, {512, 460, 5}, {700, 900, 700}};
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(rate_per_us);
    Scheduler s(arena, slots, max_batch);
    std::vector<PendingReq> reqs;
    double t = 0;
    for (int i = 0; i < nreq; i++) {
        t += gap(rng);
        const Shape &sh = shapes[rng() % shapes.size()];
        PendingReq r;
        r.id = i;
        r.kind = (rng() & 1) ? REQ_CHECK : REQ_TAG;
        r.layer = ct_layer_desc{sh.M, sh.K, sh.N, 0, 0, 100 + (uint64_t)i, 1 + (uint64_t)i, 0, 0, 0, 0, 0, 0, 0, 0};
        r.arrival_us = t;
        reqs.push_back(r);
    }
    // submit in a shuffled order: the scheduler must still admit by arrival
    std::vector<PendingReq> shuffled = reqs;
    std::shuffle(shuffled.begin(), shuffled.end(), rng);
    for (auto &r : shuffled) s.submit(r);

    std::vector<InFlight> flight;
    std::vector<int> finished(nreq, 0);
    std::vector<int> slot_used(slots, 0);
    double now = 0, last_arrival = -1;
    int64_t last_id = -1;
    int64_t converted = 0, rejected = 0, batched_multi = 0;
    int max_concurrent = 0;
    while (true) {
        // complete every batch due by now
        for (size_t i = 0; i < flight.size();) {
            if (flight[i].end <= now) {
                for (auto &it : flight[i].b.items) {
                    CHECK(finished[it.req_id] == 0);
                    finished[it.req_id] = 1;
                    if (it.status == CT_OK) {
                        const Resident *r = s.resident(it.resident);
                        CHECK(r != nullptr);  // pinned: never evicted while in flight
                        CHECK(r->pins > 0);
                    }
                }
                slot_used[flight[i].b.slot] = 0;
                s.finish(flight[i].b);
                flight.erase(flight.begin() + i);
            } else {
                i++;
            }
        }
        Batch b;
        while (s.next_batch(now, b)) {
            CHECK(!b.items.empty() && (int)b.items.size() <= max_batch);
            CHECK(b.slot >= 0 && b.slot < slots && !slot_used[b.slot]);
            slot_used[b.slot] = 1;
            size_t bytes = 0;
            for (auto &it : b.items) {
                const PendingReq &r = reqs[it.req_id];
                CHECK(r.arrival_us <= now);
                // first come, first served
                CHECK(r.arrival_us > last_arrival || (r.arrival_us == last_arrival && r.id > last_id));
                last_arrival = r.arrival_us;
                last_id = r.id;
                CHECK(it.requested == r.kind);
                if (it.status == CT_ENOMEM) {
                    CHECK(footprint(r.layer) > s.arena().size());
                    rejected++;
                    continue;
                }
                CHECK(it.status == CT_OK);
                const Resident *res = s.resident(it.resident);
                CHECK(res != nullptr);
                CHECK(res->layer.M == r.layer.M && res->layer.K == r.layer.K && res->layer.N == r.layer.N);
                if (it.kind == REQ_CHECK) {
                    CHECK(r.kind == REQ_CHECK);
                    CHECK(res->ready && res->id != r.id);
                } else {
                    CHECK(res->id == r.id && !res->ready);
                    CHECK(res->layer.seed == r.layer.seed && res->layer.layer_id == r.layer.layer_id);
                    if (r.kind == REQ_CHECK) {
                        converted++;
                        // converted only when nothing of its shape is complete and resident
                        for (auto &kv : s.residents()) {
                            const Resident &o = kv.second;
                            CHECK(!(o.ready && o.layer.M == r.layer.M && o.layer.K == r.layer.K &&
                                    o.layer.N == r.layer.N));
                        }
                    }
                }
                bytes += res->bytes;
            }
            if (b.items.size() > 1) batched_multi++;
            flight.push_back({b, now + 5.0 + (double)bytes / bytes_per_us});
        }
        max_concurrent = std::max(max_concurrent, (int)flight.size());
        // memory: residents and workspaces never overlap and account for every used byte
        {
            std::vector<std::pair<size_t, size_t>> blocks;
            size_t used = 0;
            for (auto &kv : s.residents()) {
                blocks.push_back({kv.second.off, kv.second.bytes});
                used += kv.second.bytes;
                if (kv.second.work_bytes) {
                    CHECK(!kv.second.ready);
                    blocks.push_back({kv.second.work_off, kv.second.work_bytes});
                    used += kv.second.work_bytes;
                }
            }
            std::sort(blocks.begin(), blocks.end());
            for (size_t i = 0; i + 1 < blocks.size(); i++) CHECK(blocks[i].first + blocks[i].second <= blocks[i + 1].first);
            if (!blocks.empty()) CHECK(blocks.back().first + blocks.back().second <= s.arena().size());
            CHECK(used == s.arena().used());
        }
        // next event
        double next = 1e300;
        for (auto &f : flight) next = std::min(next, f.end);
        if (s.queued() > 0 && s.next_arrival() > now) next = std::min(next, s.next_arrival());
        if (next == 1e300) {
            CHECK(s.queued() == 0);  // nothing in flight and nothing admissible would be a deadlock
            break;
        }
        now = std::max(now, next);
    }
    for (int i = 0; i < nreq; i++) CHECK(finished[i] == 1);
    const SchedStats &st = s.stats();
    CHECK(st.submitted == nreq && st.finished == nreq && st.admitted == nreq);
    CHECK(st.converted == converted && st.rejected == rejected);
    CHECK(s.arena().used() == [&] { size_t u = 0; for (auto &kv : s.residents()) u += kv.second.bytes; return u; }());
    if (expect_evictions >= 0) CHECK((st.evictions > 0) == (expect_evictions > 0));
    if (expect_rejects >= 0) CHECK((st.rejected > 0) == (expect_rejects > 0));
    std::printf("ok sched %s requests=%d batches=%lld multi=%lld max_batch=%lld concurrent=%d converted=%lld "
                "evictions=%lld rejected=%lld peak=%zu\n",
                name, nreq, (long long)st.batches, (long long)batched_multi, (long long)st.max_batch, max_concurrent,
                (long long)st.converted, (long long)st.evictions, (long long)st.rejected, st.arena_peak);
}

// Request ids name resident layers: a request whose id is that of a layer
// still resident (in flight or complete) is refused with CT_EINVAL and
// changes nothing; an id becomes free again once its layer is evicted.
static void dup_scenario() {
    Scheduler s(size_t(1) << 30, 2, 8);
    auto req = [](int64_t id, int kind, int64_t M, int64_t K, int64_t N, double t) {
        PendingReq r;
        r.id = id;
        r.kind = kind;
        r.layer = ct_layer_desc{M, K, N, 0, 0, 100 + (uint64_t)id, 1 + (uint64_t)id, 0, 0, 0, 0, 0, 0, 0, 0};
        r.arrival_us = t;
        return r;
    };
    s.submit(req(5, REQ_TAG, 64, 576, 300, 0.0));
    s.submit(req(5, REQ_TAG, 40, 2100, 70, 1.0));    // same id while 5 is in flight
    s.submit(req(7, REQ_CHECK, 70, 100, 130, 2.0));  // nothing of its shape: runs as a TAG, resident as 7
    s.submit(req(7, REQ_TAG, 33, 70, 1, 3.0));       // same id as the converted check
    Batch b;
    CHECK(s.next_batch(10.0, b));
    CHECK(b.items.size() == 4);
    CHECK(b.items[0].status == CT_OK && b.items[0].resident == 5);
    CHECK(b.items[1].status == CT_EINVAL);
    CHECK(b.items[2].status == CT_OK && b.items[2].kind == REQ_TAG && b.items[2].resident == 7);
    CHECK(b.items[3].status == CT_EINVAL);
    const size_t used = s.arena().used();
    CHECK(s.resident(5) && s.resident(5)->layer.M == 64 && s.resident(5)->layer.N == 300);
    CHECK(s.resident(7) && s.resident(7)->layer.M == 70);
    s.finish(b);
    CHECK(s.resident(5)->ready && s.resident(5)->pins == 0 && s.resident(7)->ready);
    // a complete resident layer keeps its id too
    s.submit(req(5, REQ_TAG, 40, 2100, 70, 11.0));
    CHECK(s.next_batch(12.0, b));
    CHECK(b.items.size() == 1 && b.items[0].status == CT_EINVAL);
    s.finish(b);
    CHECK(s.arena().used() == used - [&] {
        size_t w = 0;
        for (const auto &kv : s.residents()) w += kv.second.work_bytes;
        return w;
    }() - layer_work_bytes(64, 576, 300) - layer_work_bytes(70, 100, 130));
    CHECK(s.stats().duplicates == 3 && s.stats().finished == 5);
    std::printf("ok sched dupes refused=%lld resident=%zu\n", (long long)s.stats().duplicates, s.residents().size());
}

// PREP requests: the dealer runs ahead of the TAG of the same layer, which
// then runs the online phase only (and waits while the PREP is in flight);
// CHECKs never see prepared layers; a dealt prepared layer is evicted only
// after every complete one.
static void prep_scenario() {
    auto req = [](int64_t id, int kind, int64_t M, int64_t K, int64_t N, uint64_t seed, uint64_t lid, double t) {
        PendingReq r;
        r.id = id;
        r.kind = kind;
        r.layer = ct_layer_desc{M, K, N, 0, 0, seed, lid, 0, 0, 0, 0, 0, 0, 0, 0};
        r.arrival_us = t;
        return r;
    };
    Scheduler s(size_t(1) << 30, 2, 8);
    Batch b, b2;
    s.submit(req(100, REQ_PREP, 64, 576, 300, 11, 21, 0.0));
    CHECK(s.next_batch(1.0, b));
    CHECK(b.items.size() == 1 && b.items[0].kind == REQ_PREP && b.items[0].resident == 100 && !b.items[0].online_only);
    const size_t work = layer_work_bytes(64, 576, 300), lay = layer_layout(64, 576, 300).total;
    CHECK(s.resident(100)->prepared && !s.resident(100)->dealt && s.arena().used() == arena_round(lay) + work);
    s.finish(b);
    CHECK(s.resident(100)->dealt && !s.resident(100)->ready && s.arena().used() == arena_round(lay));
    // its TAG takes the prepared layer over: online phase only, workspace again
    s.submit(req(1, REQ_TAG, 64, 576, 300, 11, 21, 2.0));
    CHECK(s.next_batch(3.0, b));
    CHECK(b.items.size() == 1 && b.items[0].kind == REQ_TAG && b.items[0].online_only && b.items[0].resident == 1);
    CHECK(s.resident(100) == nullptr && s.resident(1) && !s.resident(1)->prepared && s.resident(1)->work_bytes == work);
    s.finish(b);
    CHECK(s.resident(1)->ready && s.arena().used() == arena_round(lay));
    // a TAG whose PREP is still on the device waits for it
    s.submit(req(101, REQ_PREP, 70, 100, 130, 12, 22, 4.0));
    s.submit(req(2, REQ_TAG, 70, 100, 130, 12, 22, 5.0));
    CHECK(s.next_batch(6.0, b));
    CHECK(b.items.size() == 1 && b.items[0].kind == REQ_PREP);
    CHECK(!s.next_batch(6.0, b2) && s.queued() == 1);
    s.finish(b);
    CHECK(s.next_batch(7.0, b));
    CHECK(b.items.size() == 1 && b.items[0].online_only && b.items[0].resident == 2);
    s.finish(b);
    // without a PREP a TAG deals as before; a CHECK of a prepared shape does not see it
    s.submit(req(102, REQ_PREP, 40, 2100, 70, 13, 23, 8.0));
    s.submit(req(3, REQ_TAG, 33, 70, 1, 14, 24, 8.5));
    s.submit(req(4, REQ_CHECK, 40, 2100, 70, 15, 25, 9.0));
    CHECK(s.next_batch(10.0, b));
    CHECK(b.items.size() == 3 && !b.items[1].online_only && b.items[2].kind == REQ_TAG && b.items[2].resident == 4);
    s.finish(b);
    CHECK(s.resident(102)->dealt && s.resident(4)->ready);
    const SchedStats &st = s.stats();
    CHECK(st.prepared == 3 && st.online_only == 2 && st.converted == 1 && st.finished == 7);
    // eviction order: complete layers first, then the dealt prepared one
    Scheduler t(arena_round(layer_layout(64, 64, 64).total) * 2 + layer_work_bytes(64, 64, 64), 1, 1);
    t.submit(req(200, REQ_PREP, 64, 64, 64, 31, 41, 0.0));
    CHECK(t.next_batch(1.0, b)); t.finish(b);
    t.submit(req(5, REQ_TAG, 64, 64, 64, 32, 42, 2.0));
    CHECK(t.next_batch(3.0, b)); t.finish(b);
    t.submit(req(6, REQ_TAG, 64, 64, 64, 33, 43, 4.0));
    CHECK(t.next_batch(5.0, b)); t.finish(b);
    CHECK(t.resident(200) && t.resident(5) == nullptr && t.resident(6) && t.stats().evictions == 1);
    t.submit(req(7, REQ_TAG, 64, 64, 64, 34, 44, 6.0));
    CHECK(t.next_batch(7.0, b)); t.finish(b);
    CHECK(t.stats().evictions == 2 && (t.resident(200) == nullptr) != (t.resident(6) == nullptr));
    std::printf("ok sched prep prepared=%lld online_only=%lld\n", (long long)st.prepared, (long long)st.online_only);
}

int main() {
    dup_scenario();
    prep_scenario();
    for (uint64_t seed : {1, 2, 3}) arena_scenario(seed);
    // roomy arena, overload: batches fill up, several slots busy at once, no eviction
    sched_scenario("roomy", 11, size_t(1) << 40, 3, 8, 3000, 0.05, 2000.0, 0, 0);
    // tight arena: the largest shape only just fits, completed layers get evicted
    sched_scenario("tight", 12, size_t(900) << 20, 2, 4, 3000, 0.01, 2000.0, 1, 0);
    // smaller than the largest shape: those requests are rejected, the rest served
    sched_scenario("small", 13, size_t(200) << 20, 2, 4, 1500, 0.005, 2000.0, 1, 1);
    // one slot, batch of one: plain first come, first served queue
    sched_scenario("serial", 14, size_t(1) << 30, 1, 1, 800, 0.002, 1000.0, -1, 0);
    return 0;
}
