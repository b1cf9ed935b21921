// CPU test driver for the host-side code of the library, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py:
//   * the request server's scheduling core (scp_sched.hpp) against a simulated executor and a
//     simulated clock: admission under the budget and the resident-workgroup cap, FIFO order,
//     sessions and warm starts, least-recently-used eviction, staging back-pressure, timeouts,
//     cancellation, the done list and the latency quantiles;
//   * the batch planner (scp_plan.cpp) on seeded random descriptions: every node placed exactly once,
//     trajectories and consensus groups whole, wavefront alignment and the exchange flags.
// Every check failure prints its line and the harness exits with status 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../../include/scp.h"
#include "../../paper_2603_10711_amd/csrc/scp_host.hpp"
#include "../../paper_2603_10711_amd/csrc/scp_sched.hpp"

using namespace scp;

static int g_fail = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
            g_fail = 1;                                                       \
        }                                                                     \
    } while (0)

// ---------------------------------------------------------------------------------------------
// simulated executor and clock
// ---------------------------------------------------------------------------------------------
struct Sim {
    double now = 0.0;
    double step_ms = 1.0;
    int stage_cap = 1 << 30;       // admissions the executor stages per step
    int staged_this_step = 0;
    struct Flight {
        double done_at;
        std::vector<int64_t> ids;
    };
    std::vector<Flight> flights;
    int max_inflight = 2;
    std::vector<int64_t> admit_order;
    std::vector<std::pair<int64_t, long long>> warm_admits;   // (id, source node)
};

static Request make_req(int nodes, int trajs, int wgs, size_t bytes, int32_t session = -1, int gslots = 0,
                        int shape = 0) {
    Request r;
    r.session = session;
    r.L.n_nodes = nodes;
    r.L.n_traj = trajs;
    r.L.n_wg = wgs;
    r.L.n_gslots = gslots;
    r.L.models = 1;
    r.L.kmax = 4;
    r.L.traj.assign((size_t)trajs * TR_FIELDS, 0);
    for (int t = 0; t < trajs; ++t) r.L.traj[(size_t)t * TR_FIELDS + TR_OFF] = t * (nodes / trajs);
    r.model.assign(trajs, 1);
    r.horizon.assign(trajs, nodes / trajs - 1 + shape);
    r.bytes = bytes;
    return r;
}

// Invariants of the scheduler state: budget, pool ranges, running caps, session exclusivity.
static void check_invariants(const Scheduler& sc) {
    size_t bytes = 0;
    long long nodes = 0, trajs = 0, wgs = 0;
    int resident = 0;
    std::vector<std::pair<long long, long long>> ranges;
    for (const auto& kv : sc.reqs) {
        const Request& r = kv.second;
        if (!r.resident) continue;
        ++resident;
        bytes += r.bytes;
        nodes += r.L.n_nodes;
        trajs += r.L.n_traj;
        wgs += r.L.n_wg;
        ranges.push_back({r.node_off, r.node_off + r.L.n_nodes});
    }
    CHECK(bytes == sc.st.resident_bytes);
    CHECK(resident == sc.st.resident);
    CHECK(bytes <= sc.lim.budget_bytes);
    CHECK(nodes + sc.nodes.free_total() == sc.lim.max_nodes);
    CHECK(trajs + sc.trajs.free_total() == sc.lim.max_traj);
    CHECK(wgs + sc.wgs.free_total() == sc.lim.max_wg);
    std::sort(ranges.begin(), ranges.end());
    for (size_t k = 1; k < ranges.size(); ++k) CHECK(ranges[k - 1].second <= ranges[k].first);
    int run_wg = 0;
    std::set<int32_t> sessions;
    for (int64_t id : sc.running) {
        const Request& r = sc.reqs.at(id);
        run_wg += r.L.n_wg;
        CHECK(r.state == RState::Running);
        if (r.session >= 0) {
            CHECK(!sessions.count(r.session));
            sessions.insert(r.session);
        }
    }
    CHECK(run_wg <= sc.lim.wg_cap_running);
    CHECK((int)sc.running.size() <= sc.lim.max_requests);
}

// One scheduling step of the simulated server; returns the number of requests in flight or queued.
static int sim_step(Scheduler& sc, Sim& sim) {
    // results whose step completed
    std::vector<Sim::Flight> keep;
    for (auto& f : sim.flights) {
        if (f.done_at <= sim.now) {
            for (int64_t id : f.ids) {
                Request& r = sc.reqs.at(id);
                r.info.assign((size_t)r.L.n_traj * SCP_INFO_FIELDS, 1.0);
                sc.finished(id);
            }
        } else {
            keep.push_back(f);
        }
    }
    sim.flights.swap(keep);
    if ((int)sim.flights.size() < sim.max_inflight) {
        StepPlan p;
        sim.staged_this_step = 0;
        sc.plan(
            [&](Request& r, long long x1) {
                if (sim.staged_this_step >= sim.stage_cap) return false;
                ++sim.staged_this_step;
                sim.admit_order.push_back(r.id);
                if (x1 >= 0) sim.warm_admits.push_back({r.id, x1});
                return true;
            },
            p);
        if (!p.running.empty()) {
            sc.launched(p);
            sim.flights.push_back({sim.now + sim.step_ms, p.finishing});
        }
    }
    check_invariants(sc);
    int inflight = 0;
    for (auto& f : sim.flights) inflight += (int)f.ids.size();
    return (int)(sc.queue.size() + sc.running.size()) + inflight;
}

static void run_until_idle(Scheduler& sc, Sim& sim, int max_steps = 100000) {
    for (int k = 0; k < max_steps; ++k) {
        if (sim_step(sc, sim) == 0) return;
        sim.now += 0.25;
    }
    CHECK(false);   // did not drain
}

static SchedLimits limits(size_t budget, int wg_cap = 1000, int scp_iters = 4, double timeout = 0.0) {
    SchedLimits l;
    l.max_nodes = 1 << 16;
    l.max_traj = 4096;
    l.max_wg = 4096;
    l.max_span = 32;
    l.max_requests = 64;
    l.budget_bytes = budget;
    l.wg_cap_running = wg_cap;
    l.scp_iters = scp_iters;
    l.scp_per_step = 1;
    l.timeout_ms = timeout;
    return l;
}

// FIFO admission under a budget of 2.5 requests: at most two resident, all complete in order,
// the peak stays under the budget, quantiles from the simulated clock.
static void scenario_budget() {
    Sim sim;
    Scheduler sc(limits(2500), [&] { return sim.now; });
    std::vector<int64_t> ids;
    for (int k = 0; k < 10; ++k) ids.push_back(sc.submit(make_req(100, 2, 2, 1000)));
    int peak = 0;
    for (int k = 0; k < 10000; ++k) {
        const int pend = sim_step(sc, sim);
        peak = std::max(peak, sc.st.resident);
        if (pend == 0) break;
        sim.now += 0.25;
    }
    CHECK(peak <= 2);
    CHECK(sc.st.completed == 10);
    CHECK(sc.st.peak_resident_bytes <= 2500);
    CHECK(sim.admit_order == ids);
    std::vector<int64_t> done = sc.take_done();
    CHECK(done == ids);
    CHECK(sc.take_done().empty());
    std::vector<double> lat;
    for (int64_t id : ids) lat.push_back(sc.reqs.at(id).t_done - sc.reqs.at(id).t_submit);
    std::sort(lat.begin(), lat.end());
    const scp_server_stats s = sc.stats(0);
    CHECK(s.latency_ms_p50 == lat[4]);   // nearest rank: ceil(0.5 * 10) = 5th
    CHECK(s.latency_ms_p99 == lat[9]);
    CHECK(s.latency_ms_p999 == lat[9]);  // ceil(0.999 * 10) = 10th
    CHECK(std::fabs(s.solves_per_s - 10.0 / (sc.t_last_done * 1e-3)) < 1e-9);
    for (int64_t id : ids) {
        CHECK(sc.state_of(id) == SCP_REQ_DONE);
        sc.release(id);
        CHECK(sc.state_of(id) == SCP_REQ_UNKNOWN);
    }
    CHECK(sc.reqs.empty());
    std::printf("OK budget: %d steps, p50 %.2f ms, p99 %.2f ms\n", (int)sc.st.steps, s.latency_ms_p50, s.latency_ms_p99);
}

// The resident-workgroup cap and the request cap bound the running set.
static void scenario_caps() {
    Sim sim;
    SchedLimits l = limits(1 << 30, 5);
    l.max_requests = 3;
    Scheduler sc(l, [&] { return sim.now; });
    for (int k = 0; k < 8; ++k) sc.submit(make_req(64, 1, 2, 100));
    int max_run = 0;
    for (int k = 0; k < 10000; ++k) {
        const int pend = sim_step(sc, sim);
        max_run = std::max(max_run, (int)sc.running.size());
        if (pend == 0) break;
        sim.now += 0.25;
    }
    CHECK(max_run == 2);   // 2 + 2 workgroups fit the cap of 5, a third does not
    CHECK(sc.st.completed == 8);
    std::printf("OK caps\n");
}

// Sessions: a session's requests run one after the other and warm-start in place from the
// previous solution; warm states are evicted least recently used first when room is needed.
static void scenario_sessions() {
    Sim sim;
    Scheduler sc(limits(2000), [&] { return sim.now; });
    const int64_t a1 = sc.submit(make_req(100, 2, 2, 1000, 0));
    const int64_t a2 = sc.submit(make_req(100, 2, 2, 1000, 0));
    run_until_idle(sc, sim);
    CHECK(sc.reqs.at(a1).t_done <= sc.reqs.at(a2).t_done);
    CHECK(sc.st.warm_starts == 1 && sc.reqs.at(a2).warm);
    CHECK(sim.warm_admits.size() == 1 && sim.warm_admits[0].first == a2);
    CHECK(sim.warm_admits[0].second == sc.reqs.at(a2).node_off + 1);
    CHECK(sc.st.resident == 1);   // a2's solution stays resident for the session
    // session 1 fills the second slot; session 2 needs room: session 0 (least recently used) goes
    sim.now += 1.0;
    sc.submit(make_req(100, 2, 2, 1000, 1));
    run_until_idle(sc, sim);
    CHECK(sc.st.evictions == 0 && sc.st.resident == 2);
    sim.now += 1.0;
    const int64_t c1 = sc.submit(make_req(100, 2, 2, 1000, 2));
    run_until_idle(sc, sim);
    CHECK(sc.st.evictions == 1);
    CHECK(!sc.session_warm.count(0) && sc.session_warm.count(1) && sc.session_warm.count(2));
    // session 1 warm-starts, session 0 starts cold (its state was evicted)
    sim.now += 1.0;
    const int64_t b2 = sc.submit(make_req(100, 2, 2, 1000, 1));
    run_until_idle(sc, sim);
    CHECK(sc.reqs.at(b2).warm);
    sim.now += 1.0;
    const int64_t a3 = sc.submit(make_req(100, 2, 2, 1000, 0));
    run_until_idle(sc, sim);
    CHECK(!sc.reqs.at(a3).warm);
    // a different shape never warm-starts from the session's state
    sim.now += 1.0;
    const int64_t a4 = sc.submit(make_req(100, 2, 2, 1000, 0, 0, 1));
    run_until_idle(sc, sim);
    CHECK(!sc.reqs.at(a4).warm);
    (void)c1;
    std::printf("OK sessions: warm starts %lld, evictions %lld\n", (long long)sc.st.warm_starts,
                (long long)sc.st.evictions);
}

// Staging back-pressure: an executor that stages one admission per step spreads them out, in order.
static void scenario_staging() {
    Sim sim;
    sim.stage_cap = 1;
    Scheduler sc(limits(1 << 30), [&] { return sim.now; });
    std::vector<int64_t> ids;
    for (int k = 0; k < 6; ++k) ids.push_back(sc.submit(make_req(50, 1, 1, 100)));
    sim_step(sc, sim);
    CHECK(sc.running.size() == 1 && sc.queue.size() == 5);
    run_until_idle(sc, sim);
    CHECK(sim.admit_order == ids);
    CHECK(sc.st.completed == 6);
    std::printf("OK staging\n");
}

// Timeouts: requests queued behind a full budget, or running, past the limit end without a result
// and free their place.
static void scenario_timeout() {
    Sim sim;
    sim.step_ms = 4.0;
    Scheduler sc(limits(1000, 1000, 8, 10.0), [&] { return sim.now; });
    const int64_t r1 = sc.submit(make_req(100, 2, 2, 1000));   // runs 8 steps of 4 ms: past 10 ms
    const int64_t r2 = sc.submit(make_req(100, 2, 2, 1000));   // waits behind it
    run_until_idle(sc, sim);
    CHECK(sc.state_of(r1) == SCP_REQ_TIMEOUT);
    CHECK(sc.state_of(r2) == SCP_REQ_TIMEOUT);
    CHECK(sc.st.timed_out == 2 && sc.st.completed == 0);
    CHECK(sc.st.resident == 0 && sc.nodes.free_total() == sc.lim.max_nodes);
    std::vector<int64_t> done = sc.take_done();
    CHECK(done.size() == 2);
    // a fast request under the same limit completes
    sim.step_ms = 0.5;
    const int64_t r3 = sc.submit(make_req(100, 2, 2, 1000));
    run_until_idle(sc, sim);
    CHECK(sc.state_of(r3) == SCP_REQ_DONE);
    std::printf("OK timeout\n");
}

// Cancellation: queued at once, running at the next step, in flight when its results arrive.
static void scenario_cancel() {
    Sim sim;
    sim.max_inflight = 1;
    Scheduler sc(limits(2000, 1000, 6), [&] { return sim.now; });
    const int64_t r1 = sc.submit(make_req(100, 2, 2, 1000));
    const int64_t r2 = sc.submit(make_req(100, 2, 2, 1000));
    const int64_t r3 = sc.submit(make_req(100, 2, 2, 1000));
    CHECK(sc.cancel(r3));                       // queued: ends now
    CHECK(sc.state_of(r3) == SCP_REQ_CANCELLED);
    sim_step(sc, sim);                          // r1 and r2 admitted
    CHECK(sc.running.size() == 2);
    CHECK(sc.cancel(r1));                       // running: leaves at the next step
    CHECK(sc.state_of(r1) == SCP_REQ_RUNNING);
    sim.now += 1.0;
    sim_step(sc, sim);
    CHECK(sc.state_of(r1) == SCP_REQ_CANCELLED);
    CHECK(sc.running.size() == 1);
    // r2: cancel while its results are in flight
    for (int k = 0; k < 100 && !sc.reqs.at(r2).in_flight; ++k) {
        sim.now += 1.0;
        sim_step(sc, sim);
    }
    CHECK(sc.reqs.at(r2).in_flight);
    CHECK(sc.cancel(r2));
    run_until_idle(sc, sim);
    CHECK(sc.state_of(r2) == SCP_REQ_CANCELLED);
    CHECK(sc.st.cancelled == 3 && sc.st.completed == 0);
    CHECK(!sc.cancel(r2) && !sc.cancel(12345));
    CHECK(sc.st.resident == 0);
    std::printf("OK cancel\n");
}

// ---------------------------------------------------------------------------------------------
// planner on random descriptions
// ---------------------------------------------------------------------------------------------
static void scenario_planner(int cases) {
    std::mt19937 rng(20261203u);
    int persistent = 0, spanning = 0;
    for (int c = 0; c < cases; ++c) {
        const int n = 1 + (int)(rng() % 40);
        std::vector<int32_t> model(n), horizon(n), group(n, -1);
        std::vector<double> params((size_t)n * SCP_PARAM_STRIDE, 0.0);
        int t = 0, gid = 0;
        while (t < n) {
            const int m = (rng() % 2) ? SCP_MODEL_QUAD_PM : SCP_MODEL_MARS3DOF;
            const int N = 1 + (int)(rng() % ((rng() % 4) ? 70 : 300));
            int S = 1;
            if (rng() % 3 == 0) S = 1 + (int)(rng() % 20);
            for (int k = 0; k < S && t < n; ++k, ++t) {
                model[t] = m;
                horizon[t] = N;
                group[t] = S > 1 ? gid : -1;
                double* p = &params[(size_t)t * SCP_PARAM_STRIDE];
                p[SCP_P_H] = 0.1;
                p[SCP_P_DELTA] = 1.0;
                p[SCP_P_NOBS] = (double)(rng() % 9);
                p[SCP_P_UBALL] = 20.0;
            }
            ++gid;
        }
        long long rows = 0;
        for (int q = 0; q < n; ++q) rows += horizon[q] + 1;
        std::vector<double> xg((size_t)rows * SCP_MAX_NX, 0.0), ug((size_t)rows * SCP_MAX_NU, 0.0);
        scp_problem_desc d{};
        d.n_traj = n;
        d.prec = (rng() % 3) ? SCP_F32 : SCP_F64;
        d.model = model.data();
        d.horizon = horizon.data();
        d.group = group.data();
        d.params = params.data();
        d.x_guess = xg.data();
        d.u_guess = ug.data();
        const int blocks[4] = {0, 64, 128, 256};
        d.block = blocks[rng() % 4];
        d.pack = (int)(rng() % 2);
        Layout L;
        std::string err;
        const bool ok = build_layout(&d, L, err);
        if (d.prec == SCP_F64 && d.block == 256) {   // valid for the plain form, no persistent plan
            CHECK(ok && !L.persistent_ok);
            continue;
        }
        if (!ok) std::printf("rejected: %s\n", err.c_str());
        CHECK(ok);
        if (!ok) continue;
        CHECK(L.n_nodes == rows && L.P % 256 == 0 && L.P >= L.n_nodes);
        CHECK(L.total > 0 && L.o_gx <= L.total);
        if (!L.persistent_ok) continue;
        ++persistent;
        spanning += L.n_gslots > 0;
        const int B = L.block;
        const size_t nl = (size_t)L.n_wg * B;
        CHECK(L.lane.size() == nl + 3 * (size_t)L.n_wg);
        std::vector<int> seen(L.n_nodes, 0), wg_of(L.n_nodes, -1), lane_of(L.n_nodes, -1);
        for (size_t k = 0; k < nl; ++k) {
            const int g = L.lane[k];
            if (g < 0) continue;
            CHECK(g < L.n_nodes);
            if (g >= L.n_nodes) continue;
            seen[g] += 1;
            wg_of[g] = (int)(k / B);
            lane_of[g] = (int)(k % B);
        }
        for (int g = 0; g < L.n_nodes; ++g) CHECK(seen[g] == 1);
        for (int q = 0; q < n; ++q) {
            const int off = L.traj[(size_t)q * TR_FIELDS + TR_OFF], N = horizon[q];
            const int w = wg_of[off];
            bool straddles = false;
            for (int i = 0; i <= N; ++i) {
                CHECK(wg_of[off + i] == w);                    // a trajectory stays in its workgroup
                CHECK(lane_of[off + i] == lane_of[off] + i);    // on consecutive lanes
                straddles = straddles || (lane_of[off + i] / 64 != lane_of[off] / 64);
            }
            const int info = L.lane[nl + w];
            if (straddles) CHECK(info & WG_CROSS);
            // aligned packing: a unit (a lone trajectory or a whole group) of at most 64 lanes never
            // straddles a wavefront boundary
            const int gs = L.traj[(size_t)q * TR_FIELDS + TR_GSIZE];
            if (d.pack == SCP_PACK_ALIGNED && gs * (N + 1) <= 64) CHECK(!straddles);
            CHECK((info & 0xff) == model[q]);
            // a group held by one workgroup keeps its members together
            const int gf = L.traj[(size_t)q * TR_FIELDS + TR_GFIRST];
            if (!(info & WG_SPAN)) CHECK(wg_of[L.traj[(size_t)gf * TR_FIELDS + TR_OFF]] == w);
        }
    }
    CHECK(persistent > cases / 4 && spanning > 0);   // the draws exercise both plans
    std::printf("OK planner: %d cases, %d persistent, %d with spanning groups\n", cases, persistent, spanning);
}

int main(int argc, char** argv) {
    const int cases = argc > 1 ? std::atoi(argv[1]) : 400;
    scenario_budget();
    scenario_caps();
    scenario_sessions();
    scenario_staging();
    scenario_timeout();
    scenario_cancel();
    scenario_planner(cases);
    std::printf(g_fail ? "FAILED\n" : "ALL OK\n");
    return g_fail;
}
