// Host side of the request server (include/scp_serve.h): a device pool laid out like one big
// problem arena, first-fit range allocators for nodes, trajectory slots, workgroup slots and
// spanning-group slots, a FIFO of submitted requests, MPC sessions with device-resident warm
// state, and the step pipeline (stage admissions -> scatter kernel -> one persistent kernel over
// every running request -> gather kernel for the requests that finished -> copy to host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/scp.h"
#include "../../include/scp_serve.h"
#include "scp_host.hpp"
#include "scp_launch.hpp"
#include "scp_layout.hpp"

using namespace scp;

namespace {

thread_local std::string g_server_error;

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

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

  private:
    std::map<long long, long long> free_;
};

// Bytes of the pool one unit of each kind occupies (the footprint of a request).
struct Unitsz {
    size_t node, traj, wg, span;
};

Unitsz unit_sizes(size_t esz, int block) {
    Unitsz u;
    u.node = (size_t)NPLANES * esz + 4;
    u.traj = (size_t)TR_FIELDS * 4 + SCP_PARAM_STRIDE * esz + RT_FIELDS * esz + SCP_INFO_FIELDS * 8 + FL_FIELDS * 4 + 16;
    u.wg = (size_t)block * 4 + 12;
    u.span = (size_t)GX_SYNC_STRIDE * 4 + 2 * GX_MEMBERS * GX_WIDTH * esz;
    return u;
}

struct ServerLayout {
    long long P = 0;
    size_t o_traj, o_node_traj, o_lane, o_wginfo, o_wggroup, o_params, o_planes, o_rt, o_info, o_flags, o_red,
        o_gsync, o_gx, o_in, o_out, total;
    size_t in_cap, out_cap;
};

bool valid_config(const scp_server_config* c, std::string& err) {
    if (!c) { err = "config is NULL"; return false; }
    if (c->prec != SCP_F32 && c->prec != SCP_F64) { err = "invalid precision"; return false; }
    if (c->block != 64 && c->block != 128 && c->block != 256) { err = "block must be 64, 128 or 256"; return false; }
    if (c->prec == SCP_F64 && c->block == 256) { err = "FP64 supports blocks of 64 or 128 lanes"; return false; }
    if (c->pack != SCP_PACK_ALIGNED && c->pack != SCP_PACK_DENSE) { err = "invalid pack"; return false; }
    if (c->max_nodes < 1 || c->max_nodes > (1LL << 30) || c->max_traj < 1 || c->max_wg < 1 || c->max_span < 0 ||
        c->max_requests < 1) {
        err = "capacities must be positive (max_span >= 0)";
        return false;
    }
    const scp_params& q = c->solve;
    if (!(q.admm.rho_eq > 0) || !(q.admm.rho_dyn > 0) || !(q.admm.rho_geo > 0) || q.admm.max_iters < 0 ||
        q.admm.check_every < 0 || q.scp_iters < 1) {
        err = "invalid solve parameters";
        return false;
    }
    if (c->scp_per_step < 1 || q.scp_iters % c->scp_per_step != 0) { err = "scp_per_step must divide scp_iters"; return false; }
    if (q.rho_final != 0.0 || q.adapt_mu != 0.0) {
        err = "the server runs fixed penalties (rho_final = 0, adapt_mu = 0)";
        return false;
    }
    if (c->max_inflight < 1 || c->max_inflight > 8) { err = "max_inflight must be in 1..8"; return false; }
    return true;
}

ServerLayout server_layout(const scp_server_config* c) {
    ServerLayout S;
    const size_t esz = c->prec == SCP_F32 ? 4 : 8;
    S.P = (c->max_nodes + 255) / 256 * 256;
    // staging: the largest admission the pool can hold per step, and the largest collection
    S.in_cap = align_up((size_t)c->max_traj * (TR_FIELDS * 4 + SCP_PARAM_STRIDE * esz) +
                        (size_t)c->max_nodes * (4 + (SCP_MAX_NX + SCP_MAX_NU) * esz) +
                        (size_t)c->max_wg * ((size_t)c->block * 4 + 12 + 4) + (size_t)c->max_requests * (sizeof(AdmitRec) + 64 * 4) +
                        4096);
    S.out_cap = align_up((size_t)c->max_traj * SCP_INFO_FIELDS * 8 + (size_t)c->max_nodes * (SCP_MAX_NX + SCP_MAX_NU) * esz +
                         (size_t)c->max_requests * (sizeof(CollectRec) + 64) + 4096);
    size_t o = 0;
    S.o_traj = o; o = align_up(o + (size_t)c->max_traj * TR_FIELDS * 4);
    S.o_node_traj = o; o = align_up(o + (size_t)S.P * 4);
    S.o_lane = o; o = align_up(o + (size_t)c->max_wg * c->block * 4);
    S.o_wginfo = o; o = align_up(o + (size_t)c->max_wg * 4);
    S.o_wggroup = o; o = align_up(o + (size_t)c->max_wg * 8);
    S.o_params = o; o = align_up(o + (size_t)c->max_traj * SCP_PARAM_STRIDE * esz);
    S.o_planes = o; o = align_up(o + (size_t)NPLANES * S.P * esz);
    S.o_rt = o; o = align_up(o + (size_t)c->max_traj * RT_FIELDS * esz);
    S.o_info = o; o = align_up(o + (size_t)c->max_traj * SCP_INFO_FIELDS * 8);
    S.o_flags = o; o = align_up(o + (size_t)c->max_traj * FL_FIELDS * 4);
    S.o_red = o; o = align_up(o + (size_t)c->max_traj * 2 * 8);
    S.o_gsync = o; o = align_up(o + (size_t)std::max(1, c->max_span) * GX_SYNC_STRIDE * 4);
    S.o_gx = o; o = align_up(o + (size_t)std::max(1, c->max_span) * 2 * GX_MEMBERS * GX_WIDTH * esz);
    S.o_in = o; o = align_up(o + S.in_cap);
    S.o_out = o; o = align_up(o + S.out_cap);
    S.total = o;
    return S;
}

enum class RState { Queued, Running, Done };

struct Request {
    int64_t id = 0;
    int32_t session = -1;
    // copy of the description
    std::vector<int32_t> model, horizon, group;
    std::vector<double> params, xg, ug;
    scp_problem_desc desc{};
    Layout L;           // request-local plan (offsets from 0)
    size_t bytes = 0;   // footprint
    // placement in the pool (valid while resident)
    bool resident = false;
    long long node_off = 0;
    int traj_first = 0, wg_first = 0;
    std::vector<int> gslots;
    // progress
    RState state = RState::Queued;
    uint32_t flags = 0;  // SCP_SUBMIT_*
    int scp_enq = 0;
    bool warm = false;
    double t_submit = 0, t_done = 0;
    double last_use = 0;
    // results (host, doubles)
    std::vector<double> info, x, u;
};

struct StepRec {
    hipEvent_t ev = nullptr;
    int slot = 0;                     // pinned staging slot
    std::vector<int64_t> finishing;   // requests collected in this step
    std::vector<long long> out_off;   // their offsets in the output staging
};

}  // namespace

struct scp_server {
    scp_server_config cfg;
    ServerLayout S;
    Unitsz us;
    size_t esz = 4;
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    Dev<float> df;
    Dev<double> dd;
    RangeAlloc nodes, trajs, wgs;
    std::vector<int> span_free;
    int wg_cap_running = 0;       // workgroups one launch keeps resident at one wave per SIMD
    // requests
    int64_t next_id = 1;
    std::unordered_map<int64_t, Request> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> running;
    std::unordered_map<int32_t, int64_t> session_last;   // session -> last admitted request
    std::unordered_map<int32_t, int64_t> session_warm;   // session -> resident finished request
    // pipeline
    std::vector<unsigned char*> pin_in, pin_out;          // pinned host staging, one per slot
    std::vector<bool> slot_busy;
    std::deque<StepRec> inflight;
    scp_server_stats st{};
    std::string err;

    ~scp_server() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto& r : inflight)
            if (r.ev) (void)hipEventDestroy(r.ev);
        for (auto* p : pin_in)
            if (p) (void)hipHostFree(p);
        for (auto* p : pin_out)
            if (p) (void)hipHostFree(p);
    }
};

namespace {

template <class T>
Dev<T> server_dev(const scp_server* s) {
    Dev<T> dv{};
    char* b = s->arena;
    const ServerLayout& S = s->S;
    dv.traj = reinterpret_cast<const int*>(b + S.o_traj);
    dv.node_traj = reinterpret_cast<const int*>(b + S.o_node_traj);
    dv.lane_node = reinterpret_cast<const int*>(b + S.o_lane);
    dv.params = reinterpret_cast<const T*>(b + S.o_params);
    dv.planes = reinterpret_cast<T*>(b + S.o_planes);
    dv.rt = reinterpret_cast<T*>(b + S.o_rt);
    dv.info = reinterpret_cast<double*>(b + S.o_info);
    dv.flags = reinterpret_cast<int*>(b + S.o_flags);
    dv.red = reinterpret_cast<unsigned long long*>(b + S.o_red);
    dv.n_traj = s->cfg.max_traj;
    dv.P = (int)S.P;
    dv.n_nodes = (int)s->cfg.max_nodes;
    dv.n_groups = 0;
    dv.groups = nullptr;
    dv.wg_list = nullptr;
    dv.wg_info = reinterpret_cast<const int*>(b + S.o_wginfo);
    dv.wg_group = reinterpret_cast<const int*>(b + S.o_wggroup);
    dv.gsync = reinterpret_cast<unsigned*>(b + S.o_gsync);
    dv.gx = reinterpret_cast<T*>(b + S.o_gx);
    dv.n_gslots = s->cfg.max_span;
    return dv;
}

scp_status fail(scp_server* s, scp_status st, const std::string& m) {
    if (s) s->err = m;
    return st;
}

// Request-local plan with the server's workgroup size and packing.
bool plan_request(const scp_server* s, const scp_problem_desc* d, Layout& L, std::string& err) {
    scp_problem_desc q = *d;
    q.prec = s->cfg.prec;
    q.block = s->cfg.block;
    q.pack = s->cfg.pack;
    if (!build_layout(&q, L, err)) return false;
    if (!L.persistent_ok) {
        err = (L.models & (4 | 8)) ? "the server runs the point-mass quadrotor and 3-DOF powered-descent models only"
                             : "request does not fit the server's workgroups (longest trajectory, or a group over 64 members)";
        return false;
    }
    if (L.n_wg > s->wg_cap_running) {
        err = "request needs more workgroups than one launch keeps resident";
        return false;
    }
    return true;
}

size_t request_bytes(const scp_server* s, const Layout& L) {
    return (size_t)L.n_nodes * s->us.node + (size_t)L.n_traj * s->us.traj + (size_t)L.n_wg * s->us.wg +
           (size_t)L.n_gslots * s->us.span;
}

bool same_shape(const Request& a, const Request& b) {
    return a.model == b.model && a.horizon == b.horizon && a.L.n_wg == b.L.n_wg && a.L.n_gslots == b.L.n_gslots &&
           a.L.n_nodes == b.L.n_nodes;
}

void release_placement(scp_server* s, Request& r) {
    if (!r.resident) return;
    s->nodes.release(r.node_off, r.L.n_nodes);
    s->trajs.release(r.traj_first, r.L.n_traj);
    s->wgs.release(r.wg_first, r.L.n_wg);
    for (int g : r.gslots) s->span_free.push_back(g);
    r.gslots.clear();
    r.resident = false;
    s->st.resident -= 1;
    s->st.resident_bytes -= r.bytes;
}

bool take_placement(scp_server* s, Request& r) {
    if ((int)s->span_free.size() < r.L.n_gslots) return false;
    const long long n = s->nodes.alloc(r.L.n_nodes);
    if (n < 0) return false;
    const long long t = s->trajs.alloc(r.L.n_traj);
    if (t < 0) {
        s->nodes.release(n, r.L.n_nodes);
        return false;
    }
    const long long w = s->wgs.alloc(r.L.n_wg);
    if (w < 0) {
        s->nodes.release(n, r.L.n_nodes);
        s->trajs.release(t, r.L.n_traj);
        return false;
    }
    r.node_off = n;
    r.traj_first = (int)t;
    r.wg_first = (int)w;
    r.gslots.clear();
    for (int k = 0; k < r.L.n_gslots; ++k) {
        r.gslots.push_back(s->span_free.back());
        s->span_free.pop_back();
    }
    r.resident = true;
    s->st.resident += 1;
    s->st.resident_bytes += r.bytes;
    s->st.peak_resident_bytes = std::max(s->st.peak_resident_bytes, s->st.resident_bytes);
    return true;
}

// Drop the warm state of the least recently used idle session.
bool evict_one(scp_server* s) {
    int32_t victim = -1;
    double oldest = 0;
    for (auto& kv : s->session_warm) {
        const Request& r = s->reqs.at(kv.second);
        if (victim < 0 || r.last_use < oldest) {
            victim = kv.first;
            oldest = r.last_use;
        }
    }
    if (victim < 0) return false;
    const int64_t id = s->session_warm[victim];
    s->session_warm.erase(victim);
    Request& r = s->reqs.at(id);
    release_placement(s, r);
    if (r.info.empty() && r.state == RState::Done) s->reqs.erase(id);  // already collected
    s->st.evictions += 1;
    return true;
}

int running_wgs(const scp_server* s) {
    int n = 0;
    for (int64_t id : s->running) n += s->reqs.at(id).L.n_wg;
    return n;
}

// Staged admission of one request into the blob; returns false if the blob is full.
template <class T>
bool stage_admit(scp_server* s, Request& r, unsigned char* blob, size_t& used, std::vector<AdmitRec>& recs,
                 long long x1_node) {
    const Layout& L = r.L;
    const int block = s->cfg.block;
    auto put = [&](const void* src, size_t n) -> int {
        const size_t o = (used + 15) / 16 * 16;
        if (o + n > s->S.in_cap) return -1;
        if (n) std::memcpy(blob + o, src, n);
        used = o + n;
        return (int)o;
    };
    const size_t used0 = used;
    // relocated trajectory records, parameters, node map, lane table, workgroup records
    std::vector<int> trec(L.traj);
    for (int t = 0; t < L.n_traj; ++t) {
        int* q = &trec[(size_t)t * TR_FIELDS];
        q[TR_OFF] += (int)r.node_off;
        q[TR_GFIRST] += r.traj_first;
    }
    std::vector<T> prm(r.params.size());
    for (size_t k = 0; k < prm.size(); ++k) prm[k] = T(r.params[k]);
    std::vector<int> nt(L.n_nodes);
    for (int k = 0; k < L.n_nodes; ++k) nt[k] = L.node_traj[k] + r.traj_first;
    const size_t nl = (size_t)L.n_wg * block;
    std::vector<int> lanes(L.lane.begin(), L.lane.begin() + nl);
    for (auto& v : lanes)
        if (v >= 0) v += (int)r.node_off;
    std::vector<int> wi(L.lane.begin() + nl, L.lane.begin() + nl + L.n_wg);
    std::vector<int> wgp(L.lane.begin() + nl + L.n_wg, L.lane.begin() + nl + 3 * L.n_wg);
    for (int w = 0; w < L.n_wg; ++w)
        if (wi[w] & WG_SPAN) wgp[2 * w] = r.gslots[wgp[2 * w]];
    AdmitRec a{};
    a.traj_first = r.traj_first;
    a.n_traj = L.n_traj;
    a.node_off = (int)r.node_off;
    a.n_nodes = L.n_nodes;
    a.wg_first = r.wg_first;
    a.n_wg = L.n_wg;
    a.warm = x1_node >= 0 ? 1 : 0;
    a.x1_node = (int)std::max(0LL, x1_node);
    a.keep_xinit = (r.flags & SCP_SUBMIT_MEASURED) ? 1 : 0;
    a.o_traj = put(trec.data(), trec.size() * 4);
    a.o_params = put(prm.data(), prm.size() * sizeof(T));
    a.o_node_traj = put(nt.data(), nt.size() * 4);
    a.o_lane = put(lanes.data(), lanes.size() * 4);
    a.o_wginfo = put(wi.data(), wi.size() * 4);
    a.o_wggroup = put(wgp.data(), wgp.size() * 4);
    a.o_xg = a.o_ug = 0;
    if (!a.warm) {
        std::vector<T> xg((size_t)L.n_nodes * SCP_MAX_NX, T(0)), ug((size_t)L.n_nodes * SCP_MAX_NU, T(0));
        long long xrow = 0, urow = 0;
        for (int t = 0; t < L.n_traj; ++t) {
            const int N = L.traj[(size_t)t * TR_FIELDS + TR_N], off = L.traj[(size_t)t * TR_FIELDS + TR_OFF];
            for (int i = 0; i <= N; ++i, ++xrow)
                for (int c = 0; c < SCP_MAX_NX; ++c) xg[(size_t)(off + i) * SCP_MAX_NX + c] = T(r.xg[xrow * SCP_MAX_NX + c]);
            for (int i = 0; i < N; ++i, ++urow)
                for (int c = 0; c < SCP_MAX_NU; ++c) ug[(size_t)(off + i) * SCP_MAX_NU + c] = T(r.ug[urow * SCP_MAX_NU + c]);
        }
        a.o_xg = put(xg.data(), xg.size() * sizeof(T));
        a.o_ug = put(ug.data(), ug.size() * sizeof(T));
        if (a.o_xg < 0 || a.o_ug < 0) {
            used = used0;
            return false;
        }
    }
    if (a.o_traj < 0 || a.o_params < 0 || a.o_node_traj < 0 || a.o_lane < 0 || a.o_wginfo < 0 || a.o_wggroup < 0) {
        used = used0;
        return false;
    }
    recs.push_back(a);
    return true;
}

// Move finished steps' results to their requests.
void drain(scp_server* s, bool wait_one) {
    while (!s->inflight.empty()) {
        StepRec& sr = s->inflight.front();
        hipError_t q = wait_one ? hipEventSynchronize(sr.ev) : hipEventQuery(sr.ev);
        wait_one = false;
        if (q == hipErrorNotReady) break;
        const double t = now_ms();
        const size_t esz = s->esz;
        for (size_t k = 0; k < sr.finishing.size(); ++k) {
            Request& r = s->reqs.at(sr.finishing[k]);
            const unsigned char* o = s->pin_out[sr.slot] + sr.out_off[k];
            const int nt = r.L.n_traj, nn = r.L.n_nodes;
            r.info.assign(reinterpret_cast<const double*>(o), reinterpret_cast<const double*>(o) + (size_t)nt * SCP_INFO_FIELDS);
            const unsigned char* xo = o + (size_t)nt * SCP_INFO_FIELDS * 8;
            const unsigned char* uo = xo + (size_t)nn * SCP_MAX_NX * esz;
            r.x.resize((size_t)nn * SCP_MAX_NX);
            r.u.resize((size_t)nn * SCP_MAX_NU);
            for (size_t k2 = 0; k2 < r.x.size(); ++k2)
                r.x[k2] = esz == 4 ? (double)reinterpret_cast<const float*>(xo)[k2] : reinterpret_cast<const double*>(xo)[k2];
            for (size_t k2 = 0; k2 < r.u.size(); ++k2)
                r.u[k2] = esz == 4 ? (double)reinterpret_cast<const float*>(uo)[k2] : reinterpret_cast<const double*>(uo)[k2];
            r.state = RState::Done;
            r.t_done = t;
            r.last_use = t;
            s->st.completed += 1;
            if (r.session >= 0) {
                // the solution stays resident as the session's warm state (the newest one wins)
                auto it = s->session_warm.find(r.session);
                if (it != s->session_warm.end() && it->second != r.id) {
                    Request& old = s->reqs.at(it->second);
                    release_placement(s, old);
                }
                s->session_warm[r.session] = r.id;
            } else {
                release_placement(s, r);
            }
        }
        (void)hipEventDestroy(sr.ev);
        s->slot_busy[sr.slot] = false;
        s->inflight.pop_front();
    }
}

template <class T>
scp_status do_step(scp_server* s, int wait, int32_t* pending) {
    drain(s, false);
    if ((int)s->inflight.size() >= s->cfg.max_inflight) {
        if (!wait) {
            if (pending) *pending = (int32_t)(s->queue.size() + s->running.size());
            return SCP_OK;
        }
        drain(s, true);
    }
    int slot = -1;
    for (int k = 0; k < (int)s->slot_busy.size(); ++k)
        if (!s->slot_busy[k]) {
            slot = k;
            break;
        }
    if (slot < 0) return fail(s, SCP_ERR_STATE, "no free staging slot");
    unsigned char* blob = s->pin_in[slot];
    size_t used = 0;
    std::vector<AdmitRec> recs;
    // ---- admission, FIFO; a session's requests run one after the other ----
    int run_wg = running_wgs(s);
    std::vector<int64_t> keep;
    bool blocked = false;
    std::unordered_map<int32_t, bool> session_busy;
    for (int64_t id : s->running) {
        const Request& r = s->reqs.at(id);
        if (r.session >= 0) session_busy[r.session] = true;
    }
    for (const StepRec& sr : s->inflight)
        for (int64_t id : sr.finishing) {
            const Request& r = s->reqs.at(id);
            if (r.session >= 0) session_busy[r.session] = true;   // result not drained yet
        }
    for (int64_t id : s->queue) {
        Request& r = s->reqs.at(id);
        if (blocked || (r.session >= 0 && session_busy.count(r.session))) {
            keep.push_back(id);
            if (r.session >= 0) session_busy[r.session] = true;
            continue;
        }
        if (run_wg + r.L.n_wg > s->wg_cap_running || (int)s->running.size() >= s->cfg.max_requests) {
            keep.push_back(id);
            blocked = true;
            continue;
        }
        // warm start in place from the session's resident solution
        long long x1 = -1;
        Request* prev = nullptr;
        if (r.session >= 0) {
            auto it = s->session_warm.find(r.session);
            if (it != s->session_warm.end()) {
                Request& p = s->reqs.at(it->second);
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
                auto it = s->session_warm.find(r.session);
                if (it != s->session_warm.end()) {  // different shape: the old state goes
                    release_placement(s, s->reqs.at(it->second));
                    s->session_warm.erase(it);
                }
            }
            while (!(s->st.resident_bytes + r.bytes <= s->cfg.budget_bytes && take_placement(s, r)))
                if (!evict_one(s)) break;
            placed = r.resident;
        }
        if (!placed) {
            keep.push_back(id);
            blocked = true;
            continue;
        }
        const size_t used0 = used;
        const size_t nrec0 = recs.size();
        if (!stage_admit<T>(s, r, blob, used, recs, x1)) {
            used = used0;
            recs.resize(nrec0);
            if (!prev) release_placement(s, r);
            keep.push_back(id);
            blocked = true;
            continue;
        }
        if (prev) {
            // the new request takes over the session's placement
            prev->resident = false;
            prev->gslots.clear();
            s->session_warm.erase(r.session);
            if (prev->info.empty() && prev->state == RState::Done) s->reqs.erase(prev->id);
            r.resident = true;
            s->st.warm_starts += 1;
            r.warm = true;
        }
        r.state = RState::Running;
        r.scp_enq = 0;
        s->running.push_back(id);
        run_wg += r.L.n_wg;
        if (r.session >= 0) session_busy[r.session] = true;
    }
    s->queue.assign(keep.begin(), keep.end());
    // ---- launch one step of every running request ----
    std::vector<int> wg_list;
    int models = 0, kmax = 0;
    bool span = false;
    std::vector<int64_t> finishing;
    for (int64_t id : s->running) {
        Request& r = s->reqs.at(id);
        for (int w = 0; w < r.L.n_wg; ++w) wg_list.push_back(r.wg_first + w);
        models |= r.L.models;
        kmax = std::max(kmax, r.L.kmax);
        span = span || r.L.n_gslots > 0;
        r.scp_enq += s->cfg.scp_per_step;
        if (r.scp_enq >= s->cfg.solve.scp_iters) finishing.push_back(id);
    }
    if (wg_list.empty()) {
        if (pending) *pending = (int32_t)(s->queue.size() + s->running.size());
        return SCP_OK;
    }
    // records and lists after the admission arrays
    auto put = [&](const void* src, size_t n) -> long long {
        const size_t o = (used + 15) / 16 * 16;
        if (o + n > s->S.in_cap) return -1;
        if (n) std::memcpy(blob + o, src, n);
        used = o + n;
        return (long long)o;
    };
    const long long o_recs = put(recs.data(), recs.size() * sizeof(AdmitRec));
    const long long o_list = put(wg_list.data(), wg_list.size() * 4);
    std::vector<CollectRec> crec;
    std::vector<long long> out_off;
    size_t out_used = 0;
    for (int64_t id : finishing) {
        const Request& r = s->reqs.at(id);
        const size_t o = (out_used + 15) / 16 * 16;
        const size_t n = (size_t)r.L.n_traj * SCP_INFO_FIELDS * 8 + (size_t)r.L.n_nodes * (SCP_MAX_NX + SCP_MAX_NU) * s->esz;
        crec.push_back(CollectRec{r.traj_first, r.L.n_traj, (int)r.node_off, r.L.n_nodes, (long long)o});
        out_off.push_back((long long)o);
        out_used = o + n;
    }
    const long long o_crec = put(crec.data(), crec.size() * sizeof(CollectRec));
    if (o_recs < 0 || o_list < 0 || o_crec < 0 || out_used > s->S.out_cap)
        return fail(s, SCP_ERR_STATE, "staging capacity exceeded");
    unsigned char* dev_in = reinterpret_cast<unsigned char*>(s->arena + s->S.o_in);
    unsigned char* dev_out = reinterpret_cast<unsigned char*>(s->arena + s->S.o_out);
    Dev<T> dv = server_dev<T>(s);
    dv.wg_list = reinterpret_cast<const int*>(dev_in + o_list);
    if (!span) dv.n_gslots = 0;
    KParams<T> kp{};
    const scp_params& q = s->cfg.solve;
    kp.rho_eq = T(q.admm.rho_eq);
    kp.rho_dyn = T(q.admm.rho_dyn);
    kp.rho_geo = T(q.admm.rho_geo);
    kp.eps_p = T(q.admm.eps_prim);
    kp.eps_d = T(q.admm.eps_dual);
    kp.max_iters = q.admm.max_iters;
    kp.check_every = q.admm.check_every;
    kp.eta0 = T(q.eta0);
    kp.eta1 = T(q.eta1);
    kp.eta2 = T(q.eta2);
    kp.shrink = T(q.shrink);
    kp.grow = T(q.grow);
    kp.delta_max = T(q.delta_max);
    kp.merit_w = T(q.merit_w);
    kp.rho_base[0] = q.admm.rho_eq;
    kp.rho_base[1] = q.admm.rho_dyn;
    kp.rho_base[2] = q.admm.rho_geo;
    kp.sched_s0 = 1.0;
    kp.sched_q = 1.0;
    kp.spin_ticks = group_wait_ticks(q.group_wait_ms);
    kp.n_scp = s->cfg.scp_per_step;
    kp.final_metrics = 1;
    kp.reset_info = 0;
    kp.has_groups = 1;
    hipError_t e = hipMemcpyAsync(dev_in, blob, used, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_admit<T>(dv, s->cfg.block, dev_in, (int)o_recs, (int)recs.size(), s->stream);
    if (e == hipSuccess) e = launch_persistent<T>(dv, kp, (int)wg_list.size(), s->cfg.block, models, kmax, s->stream);
    if (e == hipSuccess && !crec.empty()) {
        e = launch_collect<T>(dv, reinterpret_cast<const CollectRec*>(dev_in + o_crec), (int)crec.size(), dev_out, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s->pin_out[slot], dev_out, out_used, hipMemcpyDeviceToHost, s->stream);
    }
    StepRec sr;
    sr.slot = slot;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sr.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(sr.ev, s->stream);
    if (e != hipSuccess) return fail(s, SCP_ERR_HIP, std::string("server step: ") + hipGetErrorString(e));
    s->slot_busy[slot] = true;
    sr.finishing = finishing;
    sr.out_off = out_off;
    s->inflight.push_back(std::move(sr));
    s->st.steps += 1;
    // finishing requests leave the running set now (their collection is enqueued)
    std::vector<int64_t> still;
    for (int64_t id : s->running)
        if (std::find(finishing.begin(), finishing.end(), id) == finishing.end()) still.push_back(id);
    s->running.swap(still);
    if (pending) *pending = (int32_t)(s->queue.size() + s->running.size() + finishing.size());
    return SCP_OK;
}

}  // namespace

extern "C" {

size_t scp_server_device_bytes(const scp_server_config* cfg) {
    std::string err;
    if (!valid_config(cfg, err)) return 0;
    return server_layout(cfg).total;
}

scp_status scp_server_create(const scp_server_config* cfg, void* arena_dev, size_t arena_bytes, void* hip_stream,
                             scp_server** out) {
    g_server_error.clear();
    if (!out) {
        g_server_error = "out is NULL";
        return SCP_ERR_ARG;
    }
    *out = nullptr;
    std::string err;
    if (!valid_config(cfg, err)) {
        g_server_error = err;
        return SCP_ERR_ARG;
    }
    const ServerLayout S = server_layout(cfg);
    if (!arena_dev || arena_bytes < S.total || (reinterpret_cast<uintptr_t>(arena_dev) % kAlign) != 0) {
        g_server_error = "arena missing, too small (need " + std::to_string(S.total) + " bytes) or not 256-byte aligned";
        return SCP_ERR_ARG;
    }
    scp_server* s = new (std::nothrow) scp_server();
    if (!s) {
        g_server_error = "host allocation failed";
        return SCP_ERR_NOMEM;
    }
    s->cfg = *cfg;
    s->S = S;
    s->esz = cfg->prec == SCP_F32 ? 4 : 8;
    s->us = unit_sizes(s->esz, cfg->block);
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->arena = reinterpret_cast<char*>(arena_dev);
    s->nodes.reset(cfg->max_nodes);
    s->trajs.reset(cfg->max_traj);
    s->wgs.reset(cfg->max_wg);
    for (int g = cfg->max_span - 1; g >= 0; --g) s->span_free.push_back(g);
    // workgroups the device keeps resident at once: occupancy of the spanning-group kernel variant
    // (the largest state: both models, 8 obstacles) times the compute units; if the query fails,
    // one wave per SIMD, the LDS of the workgroup state and the device's CU count and LDS size
    s->wg_cap_running = persistent_span_resident_cap(s->esz, cfg->block, 3, 8);
    if (s->wg_cap_running <= 0) {
        int dev = 0, cus = 0, lds_cu = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
        if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
            lds_cu = 0;
        const size_t lds = std::max<size_t>(1, persistent_shared_bytes(s->esz, cfg->block));
        const int per_cu = std::max(1, std::min(4 / (cfg->block / 64), (int)((size_t)lds_cu / lds)));
        s->wg_cap_running = std::max(1, cus) * per_cu;
    }
    const int slots = cfg->max_inflight + 1;
    hipError_t e = hipSuccess;
    for (int k = 0; k < slots && e == hipSuccess; ++k) {
        void* a = nullptr;
        void* b = nullptr;
        e = hipHostMalloc(&a, S.in_cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&b, S.out_cap, hipHostMallocDefault);
        s->pin_in.push_back(reinterpret_cast<unsigned char*>(a));
        s->pin_out.push_back(reinterpret_cast<unsigned char*>(b));
        s->slot_busy.push_back(false);
    }
    // empty pool: no lanes, no trajectories
    if (e == hipSuccess) e = hipMemsetAsync(s->arena, 0, S.total, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->arena + S.o_node_traj, 0xff, (size_t)S.P * 4, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->arena + S.o_lane, 0xff, (size_t)cfg->max_wg * cfg->block * 4, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        g_server_error = std::string("server setup: ") + hipGetErrorString(e);
        delete s;
        return SCP_ERR_HIP;
    }
    *out = s;
    return SCP_OK;
}

void scp_server_destroy(scp_server* s) { delete s; }

size_t scp_server_request_bytes(const scp_server* s, const scp_problem_desc* req) {
    if (!s || !req) return 0;
    Layout L;
    std::string err;
    if (!plan_request(s, req, L, err)) return 0;
    return request_bytes(s, L);
}

scp_status scp_server_submit(scp_server* s, const scp_problem_desc* d, int32_t session, int64_t* id) {
    return scp_server_submit_ex(s, d, session, 0u, id);
}

scp_status scp_server_submit_ex(scp_server* s, const scp_problem_desc* d, int32_t session, uint32_t flags,
                                int64_t* id) {
    if (!s) return SCP_ERR_ARG;
    if (!d || !id) return fail(s, SCP_ERR_ARG, "NULL argument");
    if (flags & ~(uint32_t)SCP_SUBMIT_MEASURED) return fail(s, SCP_ERR_ARG, "unknown submission flags");
    Request r;
    std::string err;
    if (!plan_request(s, d, r.L, err)) {
        s->st.rejected += 1;
        return fail(s, SCP_ERR_ARG, err);
    }
    r.bytes = request_bytes(s, r.L);
    if (r.bytes > s->cfg.budget_bytes || r.L.n_nodes > s->cfg.max_nodes || r.L.n_traj > s->cfg.max_traj ||
        r.L.n_wg > s->cfg.max_wg || r.L.n_gslots > s->cfg.max_span) {
        s->st.rejected += 1;
        return fail(s, SCP_ERR_ARG, "request larger than the pool or the budget");
    }
    const int n = d->n_traj;
    r.model.assign(d->model, d->model + n);
    r.horizon.assign(d->horizon, d->horizon + n);
    if (d->group) r.group.assign(d->group, d->group + n);
    r.params.assign(d->params, d->params + (size_t)n * SCP_PARAM_STRIDE);
    long long xrows = 0, urows = 0;
    for (int t = 0; t < n; ++t) {
        xrows += d->horizon[t] + 1;
        urows += d->horizon[t];
    }
    r.xg.assign(d->x_guess, d->x_guess + xrows * SCP_MAX_NX);
    r.ug.assign(d->u_guess, d->u_guess + urows * SCP_MAX_NU);
    r.id = s->next_id++;
    r.session = session;
    r.flags = flags;
    r.t_submit = now_ms();
    r.last_use = r.t_submit;
    *id = r.id;
    s->queue.push_back(r.id);
    s->reqs.emplace(r.id, std::move(r));
    s->st.submitted += 1;
    return SCP_OK;
}

scp_status scp_server_step(scp_server* s, int32_t wait, int32_t* pending) {
    if (!s) return SCP_ERR_ARG;
    return s->cfg.prec == SCP_F32 ? do_step<float>(s, wait, pending) : do_step<double>(s, wait, pending);
}

scp_status scp_server_collect(scp_server* s, int64_t id, int32_t release, int32_t* state, double* latency_ms,
                              double* info, double* x, double* u) {
    if (!s) return SCP_ERR_ARG;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || (it->second.state == RState::Done && it->second.info.empty())) {
        if (state) *state = SCP_REQ_UNKNOWN;
        return SCP_OK;
    }
    Request& r = it->second;
    if (state) *state = r.state == RState::Queued ? SCP_REQ_QUEUED : r.state == RState::Running ? SCP_REQ_RUNNING : SCP_REQ_DONE;
    if (r.state != RState::Done) return SCP_OK;
    if (latency_ms) *latency_ms = r.t_done - r.t_submit;
    if (info) std::memcpy(info, r.info.data(), r.info.size() * sizeof(double));
    if (x || u) {
        // pool rows -> per-trajectory rows (N+1 states, N controls)
        long long xr = 0, ur = 0;
        for (int t = 0; t < r.L.n_traj; ++t) {
            const int N = r.L.traj[(size_t)t * TR_FIELDS + TR_N], off = r.L.traj[(size_t)t * TR_FIELDS + TR_OFF];
            for (int i = 0; i <= N; ++i, ++xr)
                if (x) std::memcpy(x + xr * SCP_MAX_NX, &r.x[(size_t)(off + i) * SCP_MAX_NX], SCP_MAX_NX * sizeof(double));
            for (int i = 0; i < N; ++i, ++ur)
                if (u) std::memcpy(u + ur * SCP_MAX_NU, &r.u[(size_t)(off + i) * SCP_MAX_NU], SCP_MAX_NU * sizeof(double));
        }
    }
    if (release) {
        r.info.clear();
        r.x.clear();
        r.u.clear();
        r.info.shrink_to_fit();
        const bool warm_holder = r.session >= 0 && s->session_warm.count(r.session) && s->session_warm[r.session] == r.id;
        if (!warm_holder && !r.resident) s->reqs.erase(it);
    }
    return SCP_OK;
}

scp_status scp_server_get_stats(const scp_server* s, scp_server_stats* out) {
    if (!s || !out) return SCP_ERR_ARG;
    *out = s->st;
    out->queued = (int32_t)s->queue.size();
    out->running = (int32_t)s->running.size();
    for (const auto& r : s->inflight) out->running += (int32_t)r.finishing.size();
    return SCP_OK;
}

const char* scp_server_last_error(const scp_server* s) {
    if (!s) return g_server_error.c_str();
    return s->err.c_str();
}

}  // extern "C"
