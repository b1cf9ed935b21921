// Host side of the request server (include/scp_serve.h): a device pool laid out like one big
// problem arena, first-fit range allocators for nodes, trajectory slots, workgroup slots and
// spanning-group slots, a FIFO of submitted requests, MPC sessions with device-resident warm
// state, and the step pipeline (stage admissions -> scatter kernel -> one persistent kernel over
// every running request -> gather kernel for the requests that finished -> copy to host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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
#include "scp_sched.hpp"
#include "scp_trace.hpp"

using namespace scp;

namespace {

thread_local std::string g_server_error;

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

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
    if (!(c->timeout_ms >= 0.0) || !std::isfinite(c->timeout_ms)) { err = "timeout_ms must be finite and >= 0"; return false; }
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
    Scheduler sched;   // admission, placement, sessions, timeouts, statistics
    // pipeline
    std::vector<unsigned char*> pin_in, pin_out;          // pinned host staging, one per slot
    std::vector<bool> slot_busy;
    std::deque<StepRec> inflight;
    std::string err;

    explicit scp_server(const SchedLimits& lim) : sched(lim, now_ms) {}
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
    if (L.n_wg > s->sched.lim.wg_cap_running) {
        err = "request needs more workgroups than one launch keeps resident";
        return false;
    }
    return true;
}

size_t request_bytes(const scp_server* s, const Layout& L) {
    return (size_t)L.n_nodes * s->us.node + (size_t)L.n_traj * s->us.traj + (size_t)L.n_wg * s->us.wg +
           (size_t)L.n_gslots * s->us.span;
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
        const size_t esz = s->esz;
        for (size_t k = 0; k < sr.finishing.size(); ++k) {
            Request& r = s->sched.reqs.at(sr.finishing[k]);
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
            s->sched.finished(r.id);
        }
        (void)hipEventDestroy(sr.ev);
        s->slot_busy[sr.slot] = false;
        s->inflight.pop_front();
    }
}

int32_t in_flight_count(const scp_server* s) {
    int32_t n = 0;
    for (const auto& r : s->inflight) n += (int32_t)r.finishing.size();
    return n;
}

template <class T>
scp_status do_step(scp_server* s, int wait, int32_t* pending) {
    TraceRange tr_step("scp_server_step");
    Scheduler& sc = s->sched;
    drain(s, false);
    if ((int)s->inflight.size() >= s->cfg.max_inflight) {
        if (!wait) {
            if (pending) *pending = (int32_t)(sc.queue.size() + sc.running.size()) + in_flight_count(s);
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
    StepPlan plan;
    {
        TraceRange tr_plan("scp_server_step: admission and staging");
        sc.plan([&](Request& r, long long x1) { return stage_admit<T>(s, r, blob, used, recs, x1); }, plan);
    }
    // ---- launch one step of every running request ----
    std::vector<int> wg_list;
    int models = 0, kmax = 0;
    bool span = false;
    for (int64_t id : plan.running) {
        const Request& r = sc.reqs.at(id);
        for (int w = 0; w < r.L.n_wg; ++w) wg_list.push_back(r.wg_first + w);
        models |= r.L.models;
        kmax = std::max(kmax, r.L.kmax);
        span = span || r.L.n_gslots > 0;
    }
    const std::vector<int64_t>& finishing = plan.finishing;
    if (wg_list.empty()) {
        if (pending) *pending = (int32_t)(sc.queue.size() + sc.running.size()) + in_flight_count(s);
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
        const Request& r = sc.reqs.at(id);
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
    kp.blowup = q.detect_blowup != 0 ? 1 : 0;
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
    // finishing requests leave the running set now (their collection is enqueued)
    sc.launched(plan);
    if (pending) *pending = (int32_t)(sc.queue.size() + sc.running.size()) + in_flight_count(s);
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
    const size_t esz = cfg->prec == SCP_F32 ? 4 : 8;
    // workgroups the device keeps resident at once: occupancy of the spanning-group kernel variant
    // (the largest state: both models, 8 obstacles) times the compute units; if the query fails,
    // one wave per SIMD, the LDS of the workgroup state and the device's CU count and LDS size
    int cap = persistent_span_resident_cap((int)esz, cfg->block, 3, 8);
    if (cap <= 0) {
        int dev = 0, cus = 0, lds_cu = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
        if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
            lds_cu = 0;
        const size_t lds = std::max<size_t>(1, persistent_shared_bytes(esz, cfg->block));
        const int per_cu = std::max(1, std::min(4 / (cfg->block / 64), (int)((size_t)lds_cu / lds)));
        cap = std::max(1, cus) * per_cu;
    }
    SchedLimits lim;
    lim.max_nodes = cfg->max_nodes;
    lim.max_traj = cfg->max_traj;
    lim.max_wg = cfg->max_wg;
    lim.max_span = cfg->max_span;
    lim.max_requests = cfg->max_requests;
    lim.budget_bytes = cfg->budget_bytes;
    lim.wg_cap_running = cap;
    lim.scp_iters = cfg->solve.scp_iters;
    lim.scp_per_step = cfg->scp_per_step;
    lim.timeout_ms = cfg->timeout_ms;
    scp_server* s = new (std::nothrow) scp_server(lim);
    if (!s) {
        g_server_error = "host allocation failed";
        return SCP_ERR_NOMEM;
    }
    s->cfg = *cfg;
    s->S = S;
    s->esz = esz;
    s->us = unit_sizes(s->esz, cfg->block);
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->arena = reinterpret_cast<char*>(arena_dev);
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
        s->sched.st.rejected += 1;
        return fail(s, SCP_ERR_ARG, err);
    }
    r.bytes = request_bytes(s, r.L);
    if (r.bytes > s->cfg.budget_bytes || r.L.n_nodes > s->cfg.max_nodes || r.L.n_traj > s->cfg.max_traj ||
        r.L.n_wg > s->cfg.max_wg || r.L.n_gslots > s->cfg.max_span) {
        s->sched.st.rejected += 1;
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
    r.session = session;
    r.flags = flags;
    *id = s->sched.submit(std::move(r));
    return SCP_OK;
}

scp_status scp_server_step(scp_server* s, int32_t wait, int32_t* pending) {
    if (!s) return SCP_ERR_ARG;
    return s->cfg.prec == SCP_F32 ? do_step<float>(s, wait, pending) : do_step<double>(s, wait, pending);
}

scp_status scp_server_collect(scp_server* s, int64_t id, int32_t release, int32_t* state, double* latency_ms,
                              double* info, double* x, double* u) {
    if (!s) return SCP_ERR_ARG;
    Scheduler& sc = s->sched;
    const int32_t stt = sc.state_of(id);
    if (state) *state = stt;
    if (stt == SCP_REQ_UNKNOWN || stt == SCP_REQ_QUEUED || stt == SCP_REQ_RUNNING) return SCP_OK;
    const Request& r = sc.reqs.at(id);
    if (latency_ms) *latency_ms = r.t_done - r.t_submit;
    if (stt == SCP_REQ_DONE) {
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
    }
    if (release) sc.release(id);
    return SCP_OK;
}

scp_status scp_server_cancel(scp_server* s, int64_t id) {
    if (!s) return SCP_ERR_ARG;
    if (!s->sched.cancel(id)) return fail(s, SCP_ERR_STATE, "no queued or running request with this id");
    return SCP_OK;
}

scp_status scp_server_take_done(scp_server* s, int64_t* ids, int32_t cap, int32_t* n) {
    if (!s || !n || cap < 0 || (cap > 0 && !ids)) return SCP_ERR_ARG;
    std::vector<int64_t>& d = s->sched.done_ids;
    const int32_t k = (int32_t)std::min<size_t>((size_t)cap, d.size());
    for (int32_t i = 0; i < k; ++i) ids[i] = d[i];
    d.erase(d.begin(), d.begin() + k);
    *n = k;
    return SCP_OK;
}

scp_status scp_server_get_stats(const scp_server* s, scp_server_stats* out) {
    if (!s || !out) return SCP_ERR_ARG;
    *out = s->sched.stats(in_flight_count(s));
    return SCP_OK;
}

const char* scp_server_last_error(const scp_server* s) {
    if (!s) return g_server_error.c_str();
    return s->err.c_str();
}

}  // extern "C"
