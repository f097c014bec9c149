// Simulated executor for the request server's admission code (rc_sched.hpp).
//
// Built and run on the CPU by tests/test_sched.py (with the address and
// undefined-behaviour sanitizers).  Requests arrive as a seeded Poisson
// process; K slots each hold one admitted round at a time, and the rounds
// share one device, which runs them one after another for overhead +
// rays / rate seconds each; library-allocated outputs are released by a
// simulated client some time after completion.  Every scenario checks:
//   - the bytes in flight never exceed the budget, and the arena never holds
//     more than is charged;
//   - requests larger than the budget are refused up front, all others
//     complete, with latency >= their round's service time;
//   - FIFO order where nothing forces backfill (plain mode, or a budget that
//     fits everything), bounded overtaking of the oldest request otherwise;
//   - after the last release the arena is one free block again and nothing is
//     charged.
// Prints one line per scenario ("name key=value ...") and "ALL OK" at the end;
// exits non-zero at the first failed check.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "rc_sched.hpp"

using rc::sched::Arena;
using rc::sched::Pending;
using rc::sched::RoundLimits;

#define CHECK(cond, ...)                                                     \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "CHECK failed at line %d: %s: ", __LINE__, #cond); \
            fprintf(stderr, __VA_ARGS__);                                    \
            fprintf(stderr, "\n");                                           \
            exit(1);                                                         \
        }                                                                    \
    } while (0)

struct SimReq {
    int id = 0;
    double arrive = 0, admit = -1, done = -1, service = 0;
    int admit_seq = -1;
    bool lib = false;
    Pending pending;
};

struct Scenario {
    const char *name;
    bool plain = false;
    int slots = 4;
    size_t budget = 1 << 30;
    int64_t max_rays = int64_t(48) << 20;
    int n = 2000;
    double rate = 2000;         // arrivals per second
    double lib_frac = 0.5;      // share of requests with library outputs
    double release_delay = 1e-3;
    double mrays_per_s = 20000;  // executor throughput
    double overhead = 2e-4;      // per round
    int max_rays_per_req = 512 * 129600;
    bool expect_fifo = false;
    int big_head_every = 0;      // every k-th request is a large one (starvation check)
    size_t big_bytes = 0;
    int refuse_every = 0;        // every k-th request is larger than the budget
};

struct Slot {
    bool busy = false;
    double until = 0;
    std::vector<SimReq *> reqs;
    size_t charged = 0;
};

static double pct(std::vector<double> v, double p)
{
    if (v.empty())
        return 0;
    std::sort(v.begin(), v.end());
    const double k = p / 100.0 * (v.size() - 1);
    const size_t lo = (size_t)k, hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (v[hi] - v[lo]) * (k - lo);
}

static void run(const Scenario &sc, unsigned seed)
{
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(sc.rate);
    std::uniform_int_distribution<int> envs(1, 512);
    std::uniform_int_distribution<int> kind(0, 2);
    std::uniform_real_distribution<double> u01(0, 1);
    const int rays_of[3] = {480 * 270, 240 * 135, 32 * 512};

    std::vector<SimReq> reqs(sc.n);
    double t = 0;
    int refused = 0;
    for (int i = 0; i < sc.n; ++i) {
        SimReq &r = reqs[i];
        r.id = i;
        t += gap(rng);
        r.arrive = t;
        const int64_t rays = (int64_t)envs(rng) * rays_of[kind(rng)];
        r.lib = u01(rng) < sc.lib_frac;
        r.pending.rays = rays;
        const size_t out = (size_t)(8 * rays);
        r.pending.arena_bytes = r.lib ? rc::sched::align_up(4 * rays) + rc::sched::align_up(4 * rays) : 0;
        r.pending.bytes = (r.lib ? r.pending.arena_bytes : out) + (size_t)(rays / 64 * 8 + 80 * 512);
        if (sc.big_head_every && i % sc.big_head_every == 0) {
            r.pending.bytes = sc.big_bytes;
            r.pending.arena_bytes = r.lib ? sc.big_bytes / 2 : 0;
        }
        if (sc.refuse_every && i % sc.refuse_every == 0)
            r.pending.bytes = sc.budget + 1;
    }

    RoundLimits lim;
    lim.budget = sc.budget;
    lim.max_rays = sc.max_rays;
    lim.fifo_only = sc.plain;
    Arena arena(sc.budget);
    size_t in_use = 0;
    std::deque<SimReq *> queue;
    std::vector<Slot> slots(sc.plain ? 1 : sc.slots);
    std::multimap<double, SimReq *> releases;  // client releases of library outputs
    int next = 0, admitted = 0, completed = 0, seq = 0, max_bypass = 0, rounds = 0;
    std::vector<double> lat;
    double now = 0, device_free = 0;
    while (true) {
        // next event
        double te = 1e300;
        if (next < sc.n)
            te = std::min(te, reqs[next].arrive);
        for (const Slot &s : slots)
            if (s.busy)
                te = std::min(te, s.until);
        if (!releases.empty())
            te = std::min(te, releases.begin()->first);
        if (te == 1e300)
            break;
        now = te;
        while (next < sc.n && reqs[next].arrive <= now) {
            SimReq &r = reqs[next++];
            if (!rc::sched::fits_alone(r.pending, lim)) {
                ++refused;
                continue;
            }
            queue.push_back(&r);
        }
        for (Slot &s : slots) {
            if (!s.busy || s.until > now)
                continue;
            for (SimReq *r : s.reqs) {
                r->done = now;
                ++completed;
                lat.push_back(r->done - r->arrive);
                CHECK(r->done - r->arrive >= r->service - 1e-12, "latency below service time (req %d)", r->id);
                if (r->lib)
                    releases.emplace(now + sc.release_delay, r);
            }
            in_use -= s.charged;
            s.charged = 0;
            s.reqs.clear();
            s.busy = false;
        }
        while (!releases.empty() && releases.begin()->first <= now) {
            SimReq *r = releases.begin()->second;
            releases.erase(releases.begin());
            arena.release(r->pending.arena_off, r->pending.arena_bytes);
            in_use -= r->pending.arena_bytes;
        }
        // admission on free slots
        for (Slot &s : slots) {
            if (s.busy || queue.empty())
                continue;
            std::vector<SimReq *> batch = rc::sched::admit(queue, in_use, arena, lim);
            if (batch.empty())
                continue;
            ++rounds;
            int64_t rays = 0;
            for (SimReq *r : batch)
                rays += r->pending.rays;
            const double service = sc.overhead + (double)rays / (sc.mrays_per_s * 1e6);
            device_free = std::max(device_free, now) + service;
            for (SimReq *r : batch) {
                r->admit = now;
                r->admit_seq = seq++;
                r->service = service;
                s.charged += r->pending.bytes - r->pending.arena_bytes;
                ++admitted;
            }
            s.reqs = batch;
            s.busy = true;
            s.until = device_free;
            CHECK(rays <= sc.max_rays || batch.size() == 1, "round over the ray cap with %zu requests", batch.size());
        }
        CHECK(in_use <= sc.budget, "in flight %zu over budget %zu", in_use, sc.budget);
        CHECK(arena.used() <= in_use, "arena holds %zu, charged %zu", arena.used(), in_use);
        for (SimReq *q : queue)
            max_bypass = std::max(max_bypass, q->pending.bypassed);
        for (const Slot &s : slots)
            for (const SimReq *r : s.reqs)
                max_bypass = std::max(max_bypass, r->pending.bypassed);
    }
    CHECK(queue.empty(), "%zu requests never admitted", queue.size());
    CHECK(completed == sc.n - refused, "completed %d of %d", completed, sc.n - refused);
    CHECK(in_use == 0, "still charged %zu", in_use);
    CHECK(arena.used() == 0 && (arena.capacity() == 0 || arena.free_blocks() == 1),
          "arena not whole again: used %zu, %zu free blocks", arena.used(), arena.free_blocks());
    CHECK(max_bypass <= lim.max_bypass, "a request was overtaken %d times (limit %d)", max_bypass, lim.max_bypass);
    if (sc.refuse_every)
        CHECK(refused == (sc.n + sc.refuse_every - 1) / sc.refuse_every, "refused %d", refused);
    else
        CHECK(refused == 0, "refused %d", refused);
    // order of admission
    std::vector<const SimReq *> by_admit;
    for (const SimReq &r : reqs)
        if (r.admit_seq >= 0)
            by_admit.push_back(&r);
    std::sort(by_admit.begin(), by_admit.end(), [](const SimReq *a, const SimReq *b) { return a->admit_seq < b->admit_seq; });
    int inversions = 0;
    for (size_t i = 1; i < by_admit.size(); ++i)
        inversions += by_admit[i]->id < by_admit[i - 1]->id;
    if (sc.expect_fifo)
        CHECK(inversions == 0, "%d admissions out of arrival order", inversions);
    printf("%s requests=%d refused=%d rounds=%d p50_ms=%.3f p99_ms=%.3f max_bypass=%d inversions=%d\n", sc.name,
           sc.n, refused, rounds, pct(lat, 50) * 1e3, pct(lat, 99) * 1e3, max_bypass, inversions);
}

static void arena_stress(unsigned seed)
{
    std::mt19937_64 rng(seed);
    const size_t cap = size_t(1) << 24;
    Arena a(cap);
    struct Blk {
        size_t off, n;
    };
    std::vector<Blk> live;
    std::uniform_int_distribution<size_t> sz(0, cap / 16);
    int fails = 0;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || (rng() & 1)) {
            const size_t n = sz(rng);
            size_t off = 0;
            if (a.alloc(n, &off)) {
                const size_t m = rc::sched::align_up(n);
                CHECK(off % rc::sched::kArenaAlign == 0 && off + m <= cap, "block [%zu, +%zu) out of range", off, m);
                for (const Blk &b : live)
                    CHECK(m == 0 || b.n == 0 || off + m <= b.off || b.off + rc::sched::align_up(b.n) <= off,
                          "block [%zu, +%zu) overlaps [%zu, +%zu)", off, m, b.off, b.n);
                live.push_back({off, n});
            } else {
                ++fails;
                CHECK(a.largest_free() < rc::sched::align_up(n), "alloc of %zu refused with %zu free in one block", n,
                      a.largest_free());
            }
        } else {
            const size_t k = rng() % live.size();
            a.release(live[k].off, live[k].n);
            live.erase(live.begin() + k);
        }
        size_t used = 0;
        for (const Blk &b : live)
            used += rc::sched::align_up(b.n);
        CHECK(a.used() == used, "arena used %zu, live %zu", a.used(), used);
    }
    for (const Blk &b : live)
        a.release(b.off, b.n);
    CHECK(a.used() == 0 && a.free_blocks() == 1 && a.largest_free() == a.capacity(), "arena not coalesced");
    printf("arena_stress ops=20000 refused=%d\n", fails);
}

int main()
{
    arena_stress(1);
    Scenario s;

    s = Scenario{"plain_fifo"};
    s.plain = true;
    s.n = 300;
    s.rate = 200;
    s.mrays_per_s = 400;
    s.expect_fifo = true;
    run(s, 2);

    s = Scenario{"batched_roomy_fifo"};  // below the executor's throughput
    s.budget = size_t(1) << 40;
    s.max_rays = int64_t(1) << 40;
    s.rate = 600;
    s.expect_fifo = true;
    run(s, 3);

    s = Scenario{"batched_stated_rate"};  // offered load above the executor's throughput
    s.n = 10000;
    s.budget = size_t(4) << 30;
    run(s, 4);

    s = Scenario{"batched_tight_budget"};
    s.budget = size_t(600) << 20;
    s.n = 3000;
    s.rate = 800;
    run(s, 5);

    s = Scenario{"batched_large_heads"};  // large requests among small ones: bounded overtaking
    s.budget = size_t(2) << 30;
    s.big_head_every = 37;
    s.big_bytes = size_t(3) << 29;
    s.n = 3000;
    s.rate = 1500;
    run(s, 6);

    s = Scenario{"batched_refusals"};
    s.budget = size_t(2) << 30;
    s.refuse_every = 9;
    s.n = 900;
    run(s, 7);

    s = Scenario{"batched_all_library_outputs"};  // arena fragmentation with slow client releases
    s.lib_frac = 1.0;
    s.release_delay = 2e-2;
    s.budget = size_t(3) << 30;
    s.n = 3000;
    run(s, 8);
    printf("ALL OK\n");
    return 0;
}
