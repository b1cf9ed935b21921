// Scheduling core of the request server (include/scp_serve.h), free of device code: the pool's
// range allocators, the FIFO of submitted requests, admission under the HBM budget and the
// resident-workgroup cap, MPC sessions with resident warm state and least-recently-used eviction,
// iteration-level step planning, request timeouts and cancellation, and the counters and latency
// quantiles of scp_server_get_stats.  The device side (staging an admission into the step's
// upload, the kernels, the result copies) lives in scp_serve.cpp; a test driver runs this core on
// the CPU against a simulated executor and clock.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/scp_serve.h"
#include "scp_host.hpp"

namespace scp {

// First-fit allocator of [0, cap) ranges with coalescing on release.
class RangeAlloc {
  public:
    explicit RangeAlloc(long long cap = 0) { reset(cap); }
    void reset(long long cap) {
        free_.clear();
        if (cap > 0) free_[0] = cap;
    }
    long long alloc(long long n) {
        if (n <= 0) return 0;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                const long long off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return off;
            }
        return -1;
    }
    void release(long long off, long long n) {
        if (n <= 0) return;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    // total free length (tests)
    long long free_total() const {
        long long n = 0;
        for (const auto& kv : free_) n += kv.second;
        return n;
    }

  private:
    std::map<long long, long long> free_;
};

enum class RState { Queued, Running, Done, Cancelled, TimedOut };

struct Request {
    int64_t id = 0;
    int32_t session = -1;
    // copy of the description
    std::vector<int32_t> model, horizon, group;
    std::vector<double> params, xg, ug;
    Layout L;           // request-local plan (offsets from 0)
    size_t bytes = 0;   // footprint
    // placement in the pool (valid while resident)
    bool resident = false;
    long long node_off = 0;
    int traj_first = 0, wg_first = 0;
    std::vector<int> gslots;
    // progress
    RState state = RState::Queued;
    uint32_t flags = 0;       // SCP_SUBMIT_*
    int scp_enq = 0;          // SCP iterations enqueued so far
    bool warm = false;
    bool in_flight = false;   // its results are being copied by a step in flight
    RState drop = RState::Queued;   // Cancelled / TimedOut requested while its results were in flight
    bool collected = false;   // results handed over and released
    double t_submit = 0, t_done = 0;
    double last_use = 0;
    // results (host, doubles)
    std::vector<double> info, x, u;
};

struct SchedLimits {
    long long max_nodes = 0;
    int max_traj = 0, max_wg = 0, max_span = 0, max_requests = 0;
    size_t budget_bytes = 0;
    int wg_cap_running = 0;   // workgroups one launch keeps resident
    int scp_iters = 1, scp_per_step = 1;
    double timeout_ms = 0.0;  // 0: none
};

// One scheduling step: the requests admitted (with the pool node of the warm-start source, -1 for
// a cold start), every running request (whose workgroups the step launches) and those among them
// that finish with this step (whose results the step collects).
struct StepPlan {
    std::vector<int64_t> admitted;
    std::vector<long long> admit_x1;
    std::vector<int64_t> running;
    std::vector<int64_t> finishing;
};

class Scheduler {
  public:
    SchedLimits lim;
    std::function<double()> clock;
    RangeAlloc nodes, trajs, wgs;
    std::vector<int> span_free;
    int64_t next_id = 1;
    std::unordered_map<int64_t, Request> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> running;
    std::unordered_map<int32_t, int64_t> session_warm;   // session -> resident finished request
    std::vector<int64_t> done_ids;                       // finished since the last take_done
    std::vector<double> latencies;                       // of completed requests (ms)
    double t_first_submit = -1.0, t_last_done = -1.0;
    scp_server_stats st{};

    Scheduler(const SchedLimits& l, std::function<double()> clk) : lim(l), clock(std::move(clk)) {
        nodes.reset(l.max_nodes);
        trajs.reset(l.max_traj);
        wgs.reset(l.max_wg);
        for (int g = l.max_span - 1; g >= 0; --g) span_free.push_back(g);
    }

    // Queue a validated request; returns its id.
    int64_t submit(Request&& r) {
        r.id = next_id++;
        r.state = RState::Queued;
        r.t_submit = clock();
        r.last_use = r.t_submit;
        if (t_first_submit < 0) t_first_submit = r.t_submit;
        const int64_t id = r.id;
        queue.push_back(id);
        reqs.emplace(id, std::move(r));
        st.submitted += 1;
        return id;
    }

    static bool same_shape(const Request& a, const Request& b) {
        return a.model == b.model && a.horizon == b.horizon && a.L.n_wg == b.L.n_wg && a.L.n_gslots == b.L.n_gslots &&
               a.L.n_nodes == b.L.n_nodes;
    }

    void release_placement(Request& r) {
        if (!r.resident) return;
        nodes.release(r.node_off, r.L.n_nodes);
        trajs.release(r.traj_first, r.L.n_traj);
        wgs.release(r.wg_first, r.L.n_wg);
        for (int g : r.gslots) span_free.push_back(g);
        r.gslots.clear();
        r.resident = false;
        st.resident -= 1;
        st.resident_bytes -= r.bytes;
    }

    bool take_placement(Request& r) {
        if ((int)span_free.size() < r.L.n_gslots) return false;
        const long long n = nodes.alloc(r.L.n_nodes);
        if (n < 0) return false;
        const long long t = trajs.alloc(r.L.n_traj);
        if (t < 0) {
            nodes.release(n, r.L.n_nodes);
            return false;
        }
        const long long w = wgs.alloc(r.L.n_wg);
        if (w < 0) {
            nodes.release(n, r.L.n_nodes);
            trajs.release(t, r.L.n_traj);
            return false;
        }
        r.node_off = n;
        r.traj_first = (int)t;
        r.wg_first = (int)w;
        r.gslots.clear();
        for (int k = 0; k < r.L.n_gslots; ++k) {
            r.gslots.push_back(span_free.back());
            span_free.pop_back();
        }
        r.resident = true;
        st.resident += 1;
        st.resident_bytes += r.bytes;
        st.peak_resident_bytes = std::max(st.peak_resident_bytes, st.resident_bytes);
        return true;
    }

    // A request nobody will collect any more can go once it holds no placement.
    void forget_if_idle(int64_t id) {
        auto it = reqs.find(id);
        if (it == reqs.end()) return;
        const Request& r = it->second;
        const bool warm_holder = r.session >= 0 && session_warm.count(r.session) && session_warm[r.session] == id;
        if (r.collected && !r.resident && !warm_holder && !r.in_flight) reqs.erase(it);
    }

    // Drop the warm state of the least recently used idle session.
    bool evict_one() {
        int32_t victim = -1;
        double oldest = 0;
        for (auto& kv : session_warm) {
            const Request& r = reqs.at(kv.second);
            if (victim < 0 || r.last_use < oldest) {
                victim = kv.first;
                oldest = r.last_use;
            }
        }
        if (victim < 0) return false;
        const int64_t id = session_warm[victim];
        session_warm.erase(victim);
        release_placement(reqs.at(id));
        forget_if_idle(id);
        st.evictions += 1;
        return true;
    }

    // End a queued or running request without a result (cancellation or timeout).
    void end_without_result(Request& r, RState why) {
        r.state = why;
        r.t_done = clock();
        release_placement(r);
        if (why == RState::Cancelled) st.cancelled += 1;
        else st.timed_out += 1;
        done_ids.push_back(r.id);
    }

    // User cancellation: a queued request leaves at once, a running one at the next step, one whose
    // results are in flight when they arrive (they are discarded).  False if the request is unknown
    // or already ended.
    bool cancel(int64_t id) {
        auto it = reqs.find(id);
        if (it == reqs.end()) return false;
        Request& r = it->second;
        if (r.state == RState::Queued) {
            queue.erase(std::find(queue.begin(), queue.end(), id));
            end_without_result(r, RState::Cancelled);
            return true;
        }
        if (r.state == RState::Running) {
            r.drop = RState::Cancelled;
            return true;
        }
        return false;
    }

    // Plan one step: timeouts and pending cancellations, then FIFO admission (a session's requests
    // run one after the other; admission stops at the first request that does not fit), then the
    // running set and the requests finishing with this step.  stage(r, x1) stages one admission
    // into the step's upload and returns false when that upload is full.
    template <class Stage>
    void plan(Stage&& stage, StepPlan& out) {
        out = StepPlan{};
        const double now = clock();
        // running requests that were cancelled or ran out of time leave before the launch
        std::vector<int64_t> still;
        for (int64_t id : running) {
            Request& r = reqs.at(id);
            RState why = r.drop;
            if (why == RState::Queued && lim.timeout_ms > 0.0 && now - r.t_submit > lim.timeout_ms) why = RState::TimedOut;
            if (why != RState::Queued) {
                r.drop = RState::Queued;
                end_without_result(r, why);
            } else {
                still.push_back(id);
            }
        }
        running.swap(still);
        if (lim.timeout_ms > 0.0) {
            std::deque<int64_t> keep;
            for (int64_t id : queue) {
                Request& r = reqs.at(id);
                if (now - r.t_submit > lim.timeout_ms) end_without_result(r, RState::TimedOut);
                else keep.push_back(id);
            }
            queue.swap(keep);
        }
        // ---- admission ----
        int run_wg = 0;
        for (int64_t id : running) run_wg += reqs.at(id).L.n_wg;
        std::unordered_map<int32_t, bool> session_busy;
        for (const auto& kv : reqs) {
            const Request& r = kv.second;
            if (r.session >= 0 && (r.state == RState::Running || r.in_flight)) session_busy[r.session] = true;
        }
        std::deque<int64_t> keep;
        bool blocked = false;
        for (int64_t id : queue) {
            Request& r = reqs.at(id);
            if (blocked || (r.session >= 0 && session_busy.count(r.session))) {
                keep.push_back(id);
                if (r.session >= 0) session_busy[r.session] = true;
                continue;
            }
            if (run_wg + r.L.n_wg > lim.wg_cap_running || (int)running.size() >= lim.max_requests) {
                keep.push_back(id);
                blocked = true;
                continue;
            }
            // warm start in place from the session's resident solution of the same shape
            long long x1 = -1;
            Request* prev = nullptr;
            if (r.session >= 0) {
                auto it = session_warm.find(r.session);
                if (it != session_warm.end()) {
                    Request& p = reqs.at(it->second);
                    if (p.resident && same_shape(p, r)) prev = &p;
                }
            }
            bool placed = false;
            if (prev) {
                r.node_off = prev->node_off;
                r.traj_first = prev->traj_first;
                r.wg_first = prev->wg_first;
                r.gslots = prev->gslots;
                x1 = prev->node_off + prev->L.traj[TR_OFF] + 1;
                placed = true;
            } else {
                if (r.session >= 0) {
                    auto it = session_warm.find(r.session);
                    if (it != session_warm.end()) {   // different shape: the old state goes
                        const int64_t old = it->second;
                        session_warm.erase(it);
                        release_placement(reqs.at(old));
                        forget_if_idle(old);
                    }
                }
                while (!(st.resident_bytes + r.bytes <= lim.budget_bytes && take_placement(r)))
                    if (!evict_one()) break;
                placed = r.resident;
            }
            if (!placed) {
                keep.push_back(id);
                blocked = true;
                continue;
            }
            if (!stage(r, x1)) {
                if (!prev) release_placement(r);
                keep.push_back(id);
                blocked = true;
                continue;
            }
            if (prev) {
                // the new request takes over the session's placement
                const int64_t pid = prev->id;
                prev->resident = false;
                prev->gslots.clear();
                session_warm.erase(r.session);
                forget_if_idle(pid);
                r.resident = true;
                st.warm_starts += 1;
                r.warm = true;
            }
            r.state = RState::Running;
            r.scp_enq = 0;
            running.push_back(id);
            out.admitted.push_back(id);
            out.admit_x1.push_back(x1);
            run_wg += r.L.n_wg;
            if (r.session >= 0) session_busy[r.session] = true;
        }
        queue.swap(keep);
        // ---- the step: every running request advances, those reaching the budget finish ----
        for (int64_t id : running) {
            Request& r = reqs.at(id);
            out.running.push_back(id);
            r.scp_enq += lim.scp_per_step;
            if (r.scp_enq >= lim.scp_iters) out.finishing.push_back(id);
        }
    }

    // The step of `p` was enqueued: its finishing requests leave the running set, their results in
    // flight.
    void launched(const StepPlan& p) {
        std::vector<int64_t> still;
        for (int64_t id : running)
            if (std::find(p.finishing.begin(), p.finishing.end(), id) == p.finishing.end()) still.push_back(id);
        running.swap(still);
        for (int64_t id : p.finishing) reqs.at(id).in_flight = true;
        st.steps += 1;
    }

    // The results of a finishing request arrived (already copied into r.info, r.x, r.u).
    void finished(int64_t id) {
        Request& r = reqs.at(id);
        r.in_flight = false;
        const double t = clock();
        if (r.drop != RState::Queued) {   // cancelled or timed out while its results were in flight
            const RState why = r.drop;
            r.drop = RState::Queued;
            r.info.clear();
            r.x.clear();
            r.u.clear();
            end_without_result(r, why);
            return;
        }
        r.state = RState::Done;
        r.t_done = t;
        r.last_use = t;
        st.completed += 1;
        latencies.push_back(t - r.t_submit);
        t_last_done = t;
        done_ids.push_back(id);
        if (r.session >= 0) {
            // the solution stays resident as the session's warm state (the newest one wins)
            auto it = session_warm.find(r.session);
            if (it != session_warm.end() && it->second != r.id) {
                const int64_t old = it->second;
                release_placement(reqs.at(old));
                session_warm.erase(it);
                forget_if_idle(old);
            }
            session_warm[r.session] = r.id;
        } else {
            release_placement(r);
        }
    }

    // Public state of a request.
    int32_t state_of(int64_t id) const {
        auto it = reqs.find(id);
        if (it == reqs.end() || it->second.collected) return SCP_REQ_UNKNOWN;
        switch (it->second.state) {
            case RState::Queued: return SCP_REQ_QUEUED;
            case RState::Running: return SCP_REQ_RUNNING;
            case RState::Done: return SCP_REQ_DONE;
            case RState::Cancelled: return SCP_REQ_CANCELLED;
            case RState::TimedOut: return SCP_REQ_TIMEOUT;
        }
        return SCP_REQ_UNKNOWN;
    }

    // Drop a request's record after its results (or its end without results) were handed over.
    void release(int64_t id) {
        auto it = reqs.find(id);
        if (it == reqs.end()) return;
        Request& r = it->second;
        r.collected = true;
        r.info.clear();
        r.x.clear();
        r.u.clear();
        r.info.shrink_to_fit();
        r.x.shrink_to_fit();
        r.u.shrink_to_fit();
        forget_if_idle(id);
    }

    // Ids of requests that ended (done, cancelled, timed out) since the last call.
    std::vector<int64_t> take_done() {
        std::vector<int64_t> out;
        out.swap(done_ids);
        return out;
    }

    // Counters, current sizes, latency quantiles (nearest rank over every completed request) and
    // the completion rate since the first submission.
    scp_server_stats stats(int32_t running_in_flight) const {
        scp_server_stats o = st;
        o.queued = (int32_t)queue.size();
        o.running = (int32_t)running.size() + running_in_flight;
        o.latency_ms_p50 = o.latency_ms_p99 = o.latency_ms_p999 = 0.0;
        if (!latencies.empty()) {
            std::vector<double> v(latencies);
            std::sort(v.begin(), v.end());
            auto q = [&](double f) {
                size_t k = (size_t)std::ceil(f * (double)v.size());
                k = std::min(std::max<size_t>(k, 1), v.size());
                return v[k - 1];
            };
            o.latency_ms_p50 = q(0.50);
            o.latency_ms_p99 = q(0.99);
            o.latency_ms_p999 = q(0.999);
        }
        o.solves_per_s = (t_last_done > t_first_submit && st.completed > 0)
                             ? (double)st.completed / ((t_last_done - t_first_submit) * 1e-3)
                             : 0.0;
        return o;
    }
};

}  // namespace scp
