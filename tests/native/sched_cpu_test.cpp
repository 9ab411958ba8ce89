// CPU test of the serving scheduler (paper_2105_04023_amd/csrc/hfr_sched.h)
// with a fake backend that answers every request with the CPU oracle's greedy
// loop (Alg. 1 with Alg. 2), built with the address/undefined-behaviour or the
// thread sanitizer by tests/test_native.py.  It checks, for many requests from
// several submitting threads over several slots:
//  - every result equals the oracle's answer for the request alone;
//  - a sketch is never used by two requests at once, and a key never has more
//    than max_copies copies resident or being built;
//  - the budget: resident + building bytes never exceed it, an oversized
//    request fails at once and evicts nothing, evictions happen under pressure;
//  - cancellation of queued requests; shutdown drains the queue.
// Exit status 0 on success; a message and status 1 on the first failure.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <thread>
#include <vector>

#include "../../paper_2105_04023_amd/csrc/hfr_sched.h"

extern "C" {
// the oracle (oracle/hfr_oracle.c), linked in
typedef struct {
    int32_t seed, rebuilt, fresh, sweeps;
    int64_t score, reach;
    double e, sigma, delta, err_l, err_g;
    int64_t visits;
} orc_step;
int orc_greedy(int64_t n, const int64_t* xadj, const int32_t* adj, const uint32_t* thr_edge, int32_t J, uint32_t seed,
               int32_t K, double eps_g, double eps_l, double eps_c, uint8_t* M, uint8_t* blk_out, orc_step* steps,
               int64_t* build_sweeps, int64_t* build_visits);
uint32_t orc_threshold(float w);
}

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "check failed: %s (%s:%d)\n", #c, __FILE__, __LINE__); \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

struct Graph {
    int64_t n;
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj;
};

// a seeded random directed graph without self-loops or duplicate edges
static Graph make_graph(int64_t n, int64_t m, uint64_t seed) {
    uint64_t s = seed * 0x9E3779B97F4A7C15ull + 1;
    auto next = [&]() {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return s;
    };
    std::vector<std::vector<char>> has(n, std::vector<char>(n, 0));
    std::vector<std::vector<int32_t>> out(n);
    for (int64_t k = 0; k < m;) {
        const int64_t u = (int64_t)(next() % n), v = (int64_t)(next() % n);
        if (u == v || has[u][v]) continue;
        has[u][v] = 1;
        out[u].push_back((int32_t)v);
        ++k;
    }
    Graph g;
    g.n = n;
    g.xadj.push_back(0);
    for (int64_t u = 0; u < n; ++u) {
        std::sort(out[u].begin(), out[u].end());
        for (int32_t v : out[u]) g.adj.push_back(v);
        g.xadj.push_back((int64_t)g.adj.size());
    }
    return g;
}

static std::vector<Graph> G;

struct Payload {
    int graph = 0;
    float p = 0.1f;
    int32_t J = 8, K = 3;
    int32_t* out = nullptr;
};

static std::vector<int32_t> oracle_seeds(const Payload& q) {
    const Graph& g = G[q.graph];
    const int64_t m = (int64_t)g.adj.size();
    std::vector<uint32_t> thr(m > 0 ? m : 1, orc_threshold(q.p));
    std::vector<uint8_t> M((size_t)g.n * q.J);
    std::vector<orc_step> st(q.K);
    int64_t bs = 0, bv = 0;
    CHECK(orc_greedy(g.n, g.xadj.data(), g.adj.data(), thr.data(), q.J, 0u, q.K, 0.01, 0.3, 0.0, M.data(), nullptr,
                     st.data(), &bs, &bv) == 0);
    std::vector<int32_t> s(q.K);
    for (int k = 0; k < q.K; ++k) s[k] = st[k].seed;
    return s;
}

// A fake sketch: remembers its key and whether a request is using it.
struct FakeSketch {
    int graph;
    float p;
    int32_t J;
    std::atomic<int> users{0};
    int slot = -1;
};

struct FakeBackend final : hfr::sched::Backend<Payload> {
    std::atomic<int> builds{0}, releases{0}, live{0};
    im_status build(int slot, const Payload& p, void** h, size_t* bytes, std::string* err) override {
        (void)err;
        auto* s = new FakeSketch;
        s->graph = p.graph;
        s->p = p.p;
        s->J = p.J;
        s->slot = slot;
        *h = s;
        *bytes = 100 * (size_t)p.J;
        builds++;
        live++;
        return IM_OK;
    }
    void adopt(int slot, void* h) override {
        auto* s = static_cast<FakeSketch*>(h);
        CHECK(s->users.load() == 0);
        s->slot = slot;
    }
    im_status select(int slot, void* h, const Payload& p, int32_t* rebuilds, std::string* err) override {
        (void)err;
        auto* s = static_cast<FakeSketch*>(h);
        CHECK(s->slot == slot);
        CHECK(s->graph == p.graph && s->p == p.p && s->J == p.J);
        CHECK(++s->users == 1);  // one request at a time
        const std::vector<int32_t> seeds = oracle_seeds(p);
        std::this_thread::sleep_for(std::chrono::microseconds(200));
        for (int k = 0; k < p.K; ++k) p.out[k] = seeds[k];
        *rebuilds = 0;
        --s->users;
        return IM_OK;
    }
    void release(void* h) override {
        auto* s = static_cast<FakeSketch*>(h);
        CHECK(s->users.load() == 0);
        delete s;
        releases++;
        live--;
    }
};

static hfr::sched::SketchKey key_of(const Payload& p) {
    uint32_t pb = 0;
    memcpy(&pb, &p.p, 4);
    return hfr::sched::SketchKey(p.graph, 0, pb, p.J, 0u, 0ull);
}

static void test_results_and_exclusivity() {
    FakeBackend be;
    hfr::sched::Scheduler<Payload> sc(4, 0, &be, 2);
    sc.start();
    const int N = 120;
    std::vector<Payload> reqs(N);
    std::vector<std::vector<int32_t>> out(N);
    std::vector<int64_t> tickets(N);
    for (int i = 0; i < N; ++i) {
        reqs[i].graph = i % (int)G.size();
        reqs[i].p = (i % 3 == 0) ? 0.3f : 0.15f;
        reqs[i].J = (i % 2) ? 8 : 16;
        reqs[i].K = 1 + i % 5;
        out[i].assign(reqs[i].K, -1);
        reqs[i].out = out[i].data();
    }
    // three submitting threads
    std::vector<std::thread> th;
    for (int t = 0; t < 3; ++t)
        th.emplace_back([&, t] {
            for (int i = t; i < N; i += 3) tickets[i] = sc.submit(key_of(reqs[i]), 1000, reqs[i]);
        });
    for (auto& x : th) x.join();
    for (int i = 0; i < N; ++i) {
        hfr::sched::Outcome o;
        CHECK(sc.wait(tickets[i], &o));
        CHECK(o.resp.status == IM_OK);
        CHECK(out[i] == oracle_seeds(reqs[i]));
    }
    const auto st = sc.stats();
    CHECK(st.completed == N && st.failed == 0);
    // 2 p values x 2 J values x graphs keys, at most 2 copies each
    CHECK(st.sketches_built <= 2 * 2 * 2 * (int64_t)G.size());
    sc.stop();
    CHECK(be.live.load() == 0 && be.builds.load() == be.releases.load());
}

static void test_budget_cancel_and_drain() {
    FakeBackend be;
    // sketches of J = 8 take 800 bytes resident and need 1000 at their peak; the budget holds two
    const size_t fixed = 5000;
    hfr::sched::Scheduler<Payload> sc(1, fixed + 2000, &be, 1);
    sc.set_fixed_bytes(fixed);
    sc.start();
    std::vector<std::vector<int32_t>> out;
    std::vector<Payload> reqs;
    for (int i = 0; i < 8; ++i) {
        Payload p;
        p.graph = i % 4;  // four keys: at most two resident, so evictions happen
        p.J = 8;
        p.K = 2;
        reqs.push_back(p);
    }
    out.resize(reqs.size());
    std::vector<int64_t> tickets;
    for (size_t i = 0; i < reqs.size(); ++i) {
        out[i].assign(reqs[i].K, -1);
        reqs[i].out = out[i].data();
        tickets.push_back(sc.submit(key_of(reqs[i]), 1000, reqs[i]));
    }
    // an oversized request fails without evicting anything
    Payload big;
    big.graph = 0;
    big.J = 16;
    std::vector<int32_t> bout(3, -1);
    big.out = bout.data();
    const int64_t tb = sc.submit(key_of(big), 3000, big);
    // cancel the last two queued requests (one slot: they have not started)
    CHECK(sc.cancel(tickets[7]) == IM_OK);
    CHECK(sc.cancel(tickets[6]) == IM_OK);
    CHECK(sc.cancel(tickets[6]) == IM_ERR_STATE);
    for (size_t i = 0; i < reqs.size(); ++i) {
        hfr::sched::Outcome o;
        CHECK(sc.wait(tickets[i], &o));
        if (i >= 6) {
            CHECK(o.resp.status == IM_ERR_STATE && out[i][0] == -1);
        } else {
            CHECK(o.resp.status == IM_OK);
            CHECK(out[i] == oracle_seeds(reqs[i]));
        }
    }
    hfr::sched::Outcome ob;
    CHECK(sc.wait(tb, &ob));
    CHECK(ob.resp.status == IM_ERR_OUT_OF_BUDGET && bout[0] == -1);
    const auto st = sc.stats();
    CHECK(st.evictions >= 2 && st.cancelled == 2);
    CHECK(st.sketch_bytes <= 2000);
    // queued work is finished by stop()
    std::vector<std::vector<int32_t>> late(5);
    std::vector<int64_t> lt;
    std::vector<Payload> lreq(5);
    for (int i = 0; i < 5; ++i) {
        lreq[i].graph = i % 2;
        lreq[i].J = 8;
        lreq[i].K = 2;
        late[i].assign(2, -1);
        lreq[i].out = late[i].data();
        lt.push_back(sc.submit(key_of(lreq[i]), 1000, lreq[i]));
    }
    sc.stop();
    for (int i = 0; i < 5; ++i) CHECK(late[i] == oracle_seeds(lreq[i]));
    CHECK(be.live.load() == 0);
}

int main() {
    for (int i = 0; i < 5; ++i) G.push_back(make_graph(20 + 3 * i, 60 + 10 * i, 100 + i));
    test_results_and_exclusivity();
    test_budget_cancel_and_drain();
    printf("sched ok\n");
    return 0;
}
