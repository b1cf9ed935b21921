// Host side of the C ABI declared in include/scp.h: problem creation and upload, the launch
// sequences of the plain and persistent forms, graph capture, the planner entry point and the
// autotuner (validation, packing and the arena layout are in scp_plan.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/scp.h"
#include "scp_host.hpp"
#include "scp_launch.hpp"
#include "scp_layout.hpp"
#include "scp_trace.hpp"

using namespace scp;

namespace {

thread_local std::string g_create_error;

const char* const kNoPersistent =
    "the persistent form needs trajectories of at most 256 nodes, consensus groups of at most 64 members and the "
    "point-mass quadrotor or 3-DOF powered-descent model, or a batch of one 6-DOF model alone with at most 64 "
    "nodes per trajectory and no consensus groups (resident ADMM); use the plain form";

}  // namespace

struct scp_problem {
    Layout L;
    scp_precision prec;
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    Dev<float> df;
    Dev<double> dd;
    bool linearized = false;
    // consensus groups spanning workgroups: workgroups the device keeps resident at once
    int span_cap = 0;
    // device whose no-allocation arena this handle holds (-1: caller arena)
    int noalloc_dev = -1;
    double lin_rho[3] = {1.0, 1.0, 1.0};
    std::string err;
    // scp_solve launch sequences captured into graphs, keyed by their parameters
    std::vector<std::pair<scp_params, hipGraphExec_t>> graphs;
    ~scp_problem() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    }
};

namespace {

// Ratio of the geometric penalty schedule (1: none).
double sched_ratio(const scp_params& s) {
    if (!(s.rho_final > 0.0) || s.scp_iters < 2) return 1.0;
    return std::pow(s.rho_final / s.admm.rho_eq, 1.0 / (double)(s.scp_iters - 1));
}

template <class T>
KParams<T> kparams(const admm_params* a, const scp_params* s) {
    KParams<T> k{};
    k.rho_eq = T(a->rho_eq);
    k.rho_dyn = T(a->rho_dyn);
    k.rho_geo = T(a->rho_geo);
    k.eps_p = T(a->eps_prim);
    k.eps_d = T(a->eps_dual);
    k.max_iters = a->max_iters;
    k.check_every = a->check_every;
    k.rho_base[0] = a->rho_eq;
    k.rho_base[1] = a->rho_dyn;
    k.rho_base[2] = a->rho_geo;
    k.sched_s0 = 1.0;
    k.sched_q = 1.0;
    k.adapt_mu = 0.0;
    k.adapt_tau = 1.0;
    k.spin_ticks = group_wait_ticks(0.0);
    if (s) {
        k.eta0 = T(s->eta0);
        k.eta1 = T(s->eta1);
        k.eta2 = T(s->eta2);
        k.shrink = T(s->shrink);
        k.grow = T(s->grow);
        k.delta_max = T(s->delta_max);
        k.merit_w = T(s->merit_w);
        k.sched_q = sched_ratio(*s);
        k.spin_ticks = group_wait_ticks(s->group_wait_ms);
        k.blowup = s->detect_blowup != 0 ? 1 : 0;
        if (s->adapt_mu > 0.0) {
            k.adapt_mu = s->adapt_mu;
            k.adapt_tau = s->adapt_tau;
        }
    }
    k.n_scp = 1;
    return k;
}

// penalties of one SCP iteration: base * factor
template <class T>
void scale_rho(KParams<T>& k, double f) {
    k.rho_eq = T(k.rho_base[0] * f);
    k.rho_dyn = T(k.rho_base[1] * f);
    k.rho_geo = T(k.rho_base[2] * f);
}

scp_status fail(scp_problem* p, scp_status st, const std::string& msg) {
    if (p) p->err = msg;
    return st;
}

scp_status hip_check(scp_problem* p, hipError_t e, const char* what) {
    if (e == hipSuccess) return SCP_OK;
    return fail(p, SCP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Checkpoint header: the arena follows it.  The fingerprint covers everything that fixes where a
// trajectory's data sits in the arena (sizes, offsets, packing tables, precision).
struct StateHeader {
    uint64_t magic;
    uint64_t fingerprint;
    uint64_t arena_bytes;
    int32_t linearized;
    int32_t prec;
    double lin_rho[3];
};
constexpr uint64_t STATE_MAGIC = 0x31544b4350435353ull;   // "SSCPCKT1"

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
    return h;
}

uint64_t layout_fingerprint(const scp_problem* p) {
    const Layout& L = p->L;
    uint64_t h = 0xcbf29ce484222325ull;
    const int64_t sizes[] = {L.n_traj, L.n_nodes, L.P, L.models, L.kmax, L.block, L.n_wg, L.n_groups,
                             (int64_t)L.esz, L.n_gslots, (int64_t)p->prec};
    h = fnv1a(h, sizes, sizeof sizes);
    const size_t offs[] = {L.o_traj, L.o_node_traj, L.o_lane, L.o_groups, L.o_params, L.o_planes, L.o_rt,
                           L.o_info, L.o_flags, L.o_red, L.o_gsync, L.o_gx, L.total};
    h = fnv1a(h, offs, sizeof offs);
    h = fnv1a(h, L.traj.data(), L.traj.size() * sizeof(int));
    h = fnv1a(h, L.node_traj.data(), L.node_traj.size() * sizeof(int));
    h = fnv1a(h, L.lane.data(), L.lane.size() * sizeof(int));
    h = fnv1a(h, L.groups.data(), L.groups.size() * sizeof(int));
    return h;
}

bool admm_valid(const admm_params* a, std::string& err) {
    if (!a) { err = "admm params NULL"; return false; }
    if (!(a->rho_eq > 0) || !(a->rho_dyn > 0) || !(a->rho_geo > 0)) { err = "penalties must be positive"; return false; }
    if (a->max_iters < 0 || a->check_every < 0) { err = "iteration counts must be >= 0"; return false; }
    return true;
}

bool same_params(const scp_params& a, const scp_params& b) {
    return a.scp_iters == b.scp_iters && a.admm.rho_eq == b.admm.rho_eq && a.admm.rho_dyn == b.admm.rho_dyn &&
           a.admm.rho_geo == b.admm.rho_geo && a.admm.max_iters == b.admm.max_iters &&
           a.admm.check_every == b.admm.check_every && a.admm.eps_prim == b.admm.eps_prim &&
           a.admm.eps_dual == b.admm.eps_dual && std::memcmp(&a.eta0, &b.eta0, sizeof(double)) == 0 &&
           a.eta1 == b.eta1 && a.eta2 == b.eta2 && a.shrink == b.shrink && a.grow == b.grow &&
           std::memcmp(&a.delta_max, &b.delta_max, sizeof(double)) == 0 && a.merit_w == b.merit_w &&
           a.form == b.form && a.scp_per_launch == b.scp_per_launch && a.rho_final == b.rho_final &&
           a.adapt_mu == b.adapt_mu && a.adapt_tau == b.adapt_tau && a.group_wait_ms == b.group_wait_ms &&
           a.lanes_per_node == b.lanes_per_node && a.detect_blowup == b.detect_blowup;
}

template <class T>
scp_status run_plain_admm(scp_problem* p, const Dev<T>& dv, const KParams<T>& kp) {
    const Layout& L = p->L;
    for (int j = 1; j <= kp.max_iters; ++j) {
        const bool check = (kp.check_every > 0 && j % kp.check_every == 0) || j == kp.max_iters;
        const int test = kp.check_every > 0 && j % kp.check_every == 0;
        hipError_t e = launch_plain<T>(PlainOp::Step1, dv, kp, L.models, L.kmax, 0, j, p->stream);
        if (e == hipSuccess) e = launch_plain<T>(PlainOp::Step234, dv, kp, L.models, L.kmax, check ? 1 : 0, j, p->stream);
        if (e == hipSuccess && check) e = launch_plain<T>(PlainOp::Resid, dv, kp, L.models, L.kmax, test, j, p->stream);
        if (e != hipSuccess) return hip_check(p, e, "ADMM kernel launch");
    }
    return SCP_OK;
}

// ADMM of a 6-DOF batch resident in one workgroup per trajectory, then the residual
// reduction of its last iteration (fixed budget)
template <class T>
scp_status run_resident_admm(scp_problem* p, const Dev<T>& dv, const KParams<T>& kp) {
    const Layout& L = p->L;
    if (kp.max_iters <= 0) return SCP_OK;
    hipError_t e = launch_resident<T>(dv, kp, L.n_traj, L.resident_block, L.models, L.kmax, p->stream);
    if (e == hipSuccess) e = launch_plain<T>(PlainOp::Resid, dv, kp, L.models, L.kmax, 0, kp.max_iters, p->stream);
    return hip_check(p, e, "resident ADMM launch");
}

template <class T>
scp_status do_linearize(scp_problem* p, const admm_params* a) {
    TraceRange tr("scp_linearize");
    const Dev<T>& dv = *reinterpret_cast<const Dev<T>*>(p->prec == SCP_F32 ? (const void*)&p->df : (const void*)&p->dd);
    KParams<T> kp = kparams<T>(a, nullptr);
    hipError_t e = launch_plain<T>(PlainOp::Lin, dv, kp, p->L.models, p->L.kmax, 0, 0, p->stream);
    return hip_check(p, e, "linearize launch");
}

template <class T>
scp_status do_admm(scp_problem* p, const admm_params* a) {
    TraceRange tr("admm_solve");
    const Dev<T>& dv = *reinterpret_cast<const Dev<T>*>(p->prec == SCP_F32 ? (const void*)&p->df : (const void*)&p->dd);
    KParams<T> kp = kparams<T>(a, nullptr);
    return run_plain_admm<T>(p, dv, kp);
}

template <class T>
scp_status do_solve(scp_problem* p, const scp_params* s) {
    TraceRange tr_solve("scp_solve");
    const Dev<T>& dv = *reinterpret_cast<const Dev<T>*>(p->prec == SCP_F32 ? (const void*)&p->df : (const void*)&p->dd);
    const Layout& L = p->L;
    KParams<T> kp = kparams<T>(&s->admm, s);
    kp.has_groups = L.n_groups > 0 ? 1 : 0;
    hipError_t e = launch_plain<T>(PlainOp::Reset, dv, kp, L.models, L.kmax, 1, 0, p->stream);
    if (e != hipSuccess) return hip_check(p, e, "reset launch");
    // lane groups of four: the 6-DOF models always, the point-mass models when asked for
    const bool resident = s->form == SCP_FORM_PERSISTENT &&
                          ((!L.persistent_ok && L.resident_ok) || (s->lanes_per_node == 4 && L.lanes4_ok));
    if (s->form == SCP_FORM_PLAIN || resident) {
        double f = 1.0;
        for (int k = 0; k < s->scp_iters; ++k, f *= kp.sched_q) {
            TraceRange tr_it(resident ? "scp_iteration (linearize, resident ADMM, accept)"
                                      : "scp_iteration (linearize, plain ADMM, accept)");
            scale_rho(kp, f);
            e = launch_plain<T>(PlainOp::Lin, dv, kp, L.models, L.kmax, 0, 0, p->stream);
            if (e != hipSuccess) return hip_check(p, e, "linearize launch");
            scp_status st = resident ? run_resident_admm<T>(p, dv, kp) : run_plain_admm<T>(p, dv, kp);
            if (st != SCP_OK) return st;
            e = launch_plain<T>(PlainOp::Accept, dv, kp, L.models, L.kmax, 0, 0, p->stream);
            if (e != hipSuccess) return hip_check(p, e, "accept launch");
        }
        e = launch_plain<T>(PlainOp::Metrics, dv, kp, L.models, L.kmax, 0, 0, p->stream);
        return hip_check(p, e, "metrics launch");
    }
    if (!L.persistent_ok)
        return fail(p, SCP_ERR_UNSUPPORTED, kNoPersistent);
    const int per = s->scp_per_launch > 0 ? s->scp_per_launch : std::max(1, s->scp_iters);
    int done = 0;
    if (s->scp_iters == 0) {
        kp.n_scp = 0;
        kp.reset_info = 1;
        kp.final_metrics = 1;
        e = launch_persistent<T>(dv, kp, L.n_wg, L.block, L.models, L.kmax, p->stream);
        return hip_check(p, e, "persistent launch");
    }
    double f = 1.0;
    while (done < s->scp_iters) {
        const int n = std::min(per, s->scp_iters - done);
        kp.n_scp = n;
        kp.sched_s0 = f;
        for (int k = 0; k < n; ++k) f *= kp.sched_q;
        kp.reset_info = done == 0 ? 1 : 0;
        kp.final_metrics = (done + n == s->scp_iters) ? 1 : 0;
        {
            TraceRange tr_it("scp_iterations (persistent launch)");
            e = launch_persistent<T>(dv, kp, L.n_wg, L.block, L.models, L.kmax, p->stream);
        }
        if (e != hipSuccess) return hip_check(p, e, "persistent launch");
        done += n;
    }
    return SCP_OK;
}

template <class T>
void stage_problem(const scp_problem_desc* d, const Layout& L, std::vector<char>& img_params, std::vector<char>& img_nom,
                   std::vector<char>& img_rt) {
    img_params.assign((size_t)L.n_traj * SCP_PARAM_STRIDE * sizeof(T), 0);
    T* prm = reinterpret_cast<T*>(img_params.data());
    for (size_t k = 0; k < (size_t)L.n_traj * SCP_PARAM_STRIDE; ++k) prm[k] = T(d->params[k]);
    // nominal planes XBAR (SCP_MAX_NX) and UBAR (SCP_MAX_NU): one contiguous block
    img_nom.assign((size_t)(SCP_MAX_NX + SCP_MAX_NU) * L.P * sizeof(T), 0);
    T* nom = reinterpret_cast<T*>(img_nom.data());
    long long xrow = 0, urow = 0;
    for (int t = 0; t < L.n_traj; ++t) {
        const int N = L.traj[(size_t)t * TR_FIELDS + TR_N], off = L.traj[(size_t)t * TR_FIELDS + TR_OFF];
        for (int i = 0; i <= N; ++i, ++xrow)
            for (int r = 0; r < SCP_MAX_NX; ++r) nom[(size_t)(PL_XBAR + r) * L.P + off + i] = T(d->x_guess[xrow * SCP_MAX_NX + r]);
        for (int i = 0; i < N; ++i, ++urow)
            for (int r = 0; r < SCP_MAX_NU; ++r) nom[(size_t)(PL_UBAR + r) * L.P + off + i] = T(d->u_guess[urow * SCP_MAX_NU + r]);
    }
    img_rt.assign((size_t)L.n_traj * RT_FIELDS * sizeof(T), 0);
    T* rt = reinterpret_cast<T*>(img_rt.data());
    for (int t = 0; t < L.n_traj; ++t) rt[t * RT_FIELDS + RT_DELTA] = T(d->params[(size_t)t * SCP_PARAM_STRIDE + SCP_P_DELTA]);
}

std::mutex g_tune_mu;
std::map<std::string, scp_tune_entry> g_tune_cache;

// Cache key of the autotuner: problem shape (precision, model, horizon, obstacle count and group
// layout of every trajectory), the solve parameters and the cadence list.
std::string tune_key(const scp_problem_desc* d, const scp_params* q, const std::vector<int>& cads) {
    std::string k = std::to_string(d->prec) + "|" + std::to_string(d->n_traj) + "|";
    for (int t = 0; t < d->n_traj; ++t) {
        const int K = (int)d->params[(size_t)t * SCP_PARAM_STRIDE + SCP_P_NOBS];
        const int same = (d->group && t > 0 && d->group[t] >= 0 && d->group[t] == d->group[t - 1]) ? 1 : 0;
        k += std::to_string(d->model[t]) + "," + std::to_string(d->horizon[t]) + "," + std::to_string(K) + "," +
             std::to_string(same) + ";";
    }
    char buf[512];
    std::snprintf(buf, sizeof buf, "|%d|%.17g,%.17g,%.17g,%d,%.17g,%.17g|%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g|%d|%.17g|%.17g,%.17g|",
                  q->scp_iters, q->admm.rho_eq, q->admm.rho_dyn, q->admm.rho_geo, q->admm.max_iters,
                  q->admm.eps_prim, q->admm.eps_dual, q->eta0, q->eta1, q->eta2, q->shrink, q->grow, q->delta_max,
                  q->merit_w, q->scp_per_launch, q->rho_final, q->adapt_mu, q->adapt_tau);
    k += buf;
    for (int c : cads) k += std::to_string(c) + ",";
    return k;
}

}  // namespace

namespace scp {

void set_create_error(const std::string& msg) { g_create_error = msg; }
void problem_mark_noalloc(scp_problem* p, int dev) { p->noalloc_dev = dev; }

}  // namespace scp

extern "C" {

size_t scp_problem_device_bytes(const scp_problem_desc* desc) {
    Layout L;
    std::string err;
    if (!build_layout(desc, L, err)) return 0;
    return L.total;
}

scp_status scp_problem_create(const scp_problem_desc* desc, void* arena_dev, size_t arena_bytes, void* hip_stream,
                              scp_problem** out) {
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return SCP_ERR_ARG;
    }
    *out = nullptr;
    scp_problem* p = new (std::nothrow) scp_problem();
    if (!p) {
        g_create_error = "host allocation failed";
        return SCP_ERR_NOMEM;
    }
    std::string err;
    if (!build_layout(desc, p->L, err)) {
        g_create_error = err;
        delete p;
        return SCP_ERR_ARG;
    }
    if (!arena_dev || arena_bytes < p->L.total || (reinterpret_cast<uintptr_t>(arena_dev) % kAlign) != 0) {
        g_create_error = "arena missing, too small (need " + std::to_string(p->L.total) + " bytes) or not 256-byte aligned";
        delete p;
        return SCP_ERR_ARG;
    }
    p->prec = desc->prec;
    p->stream = reinterpret_cast<hipStream_t>(hip_stream);
    p->arena = reinterpret_cast<char*>(arena_dev);
    const Layout& L = p->L;
    std::vector<char> img_params, img_nom, img_rt;
    if (p->prec == SCP_F32) stage_problem<float>(desc, L, img_params, img_nom, img_rt);
    else stage_problem<double>(desc, L, img_params, img_nom, img_rt);
    hipError_t e = hipMemsetAsync(p->arena, 0, L.total, p->stream);
    auto cp = [&](size_t off, const void* src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpyAsync(p->arena + off, src, n, hipMemcpyHostToDevice, p->stream);
    };
    cp(L.o_traj, L.traj.data(), L.traj.size() * 4);
    cp(L.o_node_traj, L.node_traj.data(), L.node_traj.size() * 4);
    cp(L.o_lane, L.lane.data(), L.lane.size() * 4);
    if (!L.groups.empty()) cp(L.o_groups, L.groups.data(), L.groups.size() * 4);
    cp(L.o_params, img_params.data(), img_params.size());
    cp(L.o_planes, img_nom.data(), img_nom.size());
    cp(L.o_planes + (size_t)PL_XG * L.P * L.esz, img_nom.data(), img_nom.size());   // kept for scp_reset
    cp(L.o_rt, img_rt.data(), img_rt.size());
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        g_create_error = std::string("upload failed: ") + hipGetErrorString(e);
        delete p;
        return SCP_ERR_HIP;
    }
    p->df = make_dev<float>(L, p->arena);
    p->dd = make_dev<double>(L, p->arena);
    if (L.persistent_ok && L.n_gslots > 0) p->span_cap = persistent_span_resident_cap((int)L.esz, L.block, L.models, L.kmax);
    *out = p;
    return SCP_OK;
}

void scp_problem_destroy(scp_problem* p) {
    if (p && p->noalloc_dev >= 0) noalloc_release(p->noalloc_dev);
    delete p;
}

scp_status scp_linearize(scp_problem* p, const admm_params* prm) {
    if (!p) return SCP_ERR_ARG;
    admm_params def{1.0, 1.0, 1.0, 0, 0, 0.0, 0.0};
    const admm_params* a = prm ? prm : &def;
    std::string err;
    if (!admm_valid(a, err)) return fail(p, SCP_ERR_ARG, err);
    scp_status st = p->prec == SCP_F32 ? do_linearize<float>(p, a) : do_linearize<double>(p, a);
    if (st == SCP_OK) {
        p->linearized = true;
        p->lin_rho[0] = a->rho_eq;
        p->lin_rho[1] = a->rho_dyn;
        p->lin_rho[2] = a->rho_geo;
    }
    return st;
}

scp_status admm_solve(scp_problem* p, const admm_params* prm) {
    if (!p) return SCP_ERR_ARG;
    std::string err;
    if (!admm_valid(prm, err)) return fail(p, SCP_ERR_ARG, err);
    if (!p->linearized) return fail(p, SCP_ERR_STATE, "admm_solve before scp_linearize");
    if (prm->rho_eq != p->lin_rho[0] || prm->rho_dyn != p->lin_rho[1] || prm->rho_geo != p->lin_rho[2])
        return fail(p, SCP_ERR_ARG, "penalties differ from those the factors were built with");
    return p->prec == SCP_F32 ? do_admm<float>(p, prm) : do_admm<double>(p, prm);
}

scp_status scp_solve(scp_problem* p, const scp_params* prm) {
    if (!p) return SCP_ERR_ARG;
    if (!prm) return fail(p, SCP_ERR_ARG, "scp params NULL");
    std::string err;
    if (!admm_valid(&prm->admm, err)) return fail(p, SCP_ERR_ARG, err);
    if (prm->scp_iters < 0) return fail(p, SCP_ERR_ARG, "scp_iters must be >= 0");
    if (prm->form != SCP_FORM_PLAIN && prm->form != SCP_FORM_PERSISTENT) return fail(p, SCP_ERR_ARG, "invalid form");
    if (prm->graph != 0 && prm->graph != 1) return fail(p, SCP_ERR_ARG, "graph must be 0 or 1");
    if (!(prm->rho_final >= 0.0)) return fail(p, SCP_ERR_ARG, "rho_final must be >= 0");
    if (!(prm->adapt_mu == 0.0 || (prm->adapt_mu > 1.0 && prm->adapt_tau > 1.0 && std::isfinite(prm->adapt_mu) &&
                                   std::isfinite(prm->adapt_tau))))
        return fail(p, SCP_ERR_ARG, "adaptive penalty: adapt_mu must be 0 (off) or > 1 with adapt_tau > 1");
    if (prm->adapt_mu > 0.0 && (prm->admm.check_every > 0 || p->L.n_groups > 0))
        return fail(p, SCP_ERR_UNSUPPORTED, "the adaptive penalty runs fixed budgets (check_every = 0) "
                                             "without consensus groups");
    if (prm->form == SCP_FORM_PERSISTENT && !p->L.persistent_ok && !p->L.resident_ok)
        return fail(p, SCP_ERR_UNSUPPORTED, kNoPersistent);
    if (prm->lanes_per_node != 0 && prm->lanes_per_node != 1 && prm->lanes_per_node != 4)
        return fail(p, SCP_ERR_ARG, "lanes_per_node must be 0, 1 or 4");
    if (prm->form == SCP_FORM_PERSISTENT && prm->lanes_per_node == 1 && !p->L.persistent_ok)
        return fail(p, SCP_ERR_UNSUPPORTED, "one lane per node: the fused persistent kernel does not hold this batch "
                                             "(6-DOF models, or trajectories / groups too long)");
    if (prm->form == SCP_FORM_PERSISTENT && prm->lanes_per_node == 4 && !p->L.resident_ok) {
        if (!p->L.lanes4_ok)
            return fail(p, SCP_ERR_UNSUPPORTED, "lane groups of four need trajectories of at most 64 nodes and no "
                                                 "consensus groups");
        if (prm->admm.check_every > 0)
            return fail(p, SCP_ERR_UNSUPPORTED, "lane groups of four run fixed ADMM budgets (check_every = 0)");
    }
    if (prm->form == SCP_FORM_PERSISTENT && prm->lanes_per_node != 4 && p->L.persistent_ok && p->L.n_gslots > 0 &&
        p->L.n_wg > p->span_cap)
        return fail(p, SCP_ERR_UNSUPPORTED, "consensus groups spanning several workgroups need every workgroup of "
                                             "the launch resident at once: the batch has " + std::to_string(p->L.n_wg) +
                                             " workgroups, the device keeps " + std::to_string(p->span_cap) +
                                             " resident; use the plain form or smaller batches");
    if (prm->form == SCP_FORM_PERSISTENT && !p->L.persistent_ok && prm->admm.check_every > 0)
        return fail(p, SCP_ERR_UNSUPPORTED, "the resident ADMM of 6-DOF batches runs fixed budgets "
                                             "(check_every = 0)");
    scp_status st = SCP_OK;
    if (!prm->graph) {
        st = p->prec == SCP_F32 ? do_solve<float>(p, prm) : do_solve<double>(p, prm);
    } else {
        hipGraphExec_t exec = nullptr;
        for (auto& g : p->graphs)
            if (same_params(g.first, *prm)) exec = g.second;
        if (!exec) {
            hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                (void)hipGetLastError();  // the launch checks that follow must not see this error
                return hip_check(p, e, "graph capture (the stream must not be the legacy default stream)");
            }
            st = p->prec == SCP_F32 ? do_solve<float>(p, prm) : do_solve<double>(p, prm);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(p->stream, &graph);
            if (st != SCP_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return hip_check(p, e, "graph capture");
            }
            p->graphs.emplace_back(*prm, exec);
        }
        st = hip_check(p, hipGraphLaunch(exec, p->stream), "graph launch");
    }
    if (st == SCP_OK) {
        p->linearized = false;
    }
    return st;
}

scp_status scp_reset(scp_problem* p) {
    if (!p) return SCP_ERR_ARG;
    hipError_t e;
    if (p->prec == SCP_F32) {
        KParams<float> kp{};
        e = launch_plain<float>(PlainOp::ResetState, p->df, kp, p->L.models, p->L.kmax, 1, 0, p->stream);
    } else {
        KParams<double> kp{};
        e = launch_plain<double>(PlainOp::ResetState, p->dd, kp, p->L.models, p->L.kmax, 1, 0, p->stream);
    }
    p->linearized = false;
    return hip_check(p, e, "reset launch");
}

int32_t scp_field_width(int32_t field) {
    switch (field) {
        case SCP_FIELD_XBAR: case SCP_FIELD_X: case SCP_FIELD_Z: case SCP_FIELD_LAM: case SCP_FIELD_MU:
        case SCP_FIELD_DDYN: case SCP_FIELD_D: return SCP_MAX_NX;
        case SCP_FIELD_UBAR: case SCP_FIELD_U: return SCP_MAX_NU;
        case SCP_FIELD_COPY: case SCP_FIELD_DUAL: return MAX_C;
        case SCP_FIELD_A: return SCP_MAX_NX * SCP_MAX_NX;
        case SCP_FIELD_B: return SCP_MAX_NX * SCP_MAX_NU;
        case SCP_FIELD_BOXLO: case SCP_FIELD_BOXHI: return SCP_MAX_NX + SCP_MAX_NU;
        case SCP_FIELD_HS: return 32;
        default: return 0;
    }
}

scp_status scp_get_field(const scp_problem* cp, int32_t field, void* dst_dev) {
    scp_problem* p = const_cast<scp_problem*>(cp);
    if (!p) return SCP_ERR_ARG;
    const int w = scp_field_width(field);
    if (!w || !dst_dev) return fail(p, SCP_ERR_ARG, "invalid field id or NULL destination");
    int plane = 0, mode = 0;
    switch (field) {
        case SCP_FIELD_XBAR: plane = PL_XBAR; break;
        case SCP_FIELD_UBAR: plane = PL_UBAR; break;
        case SCP_FIELD_X: plane = PL_X; break;
        case SCP_FIELD_U: plane = PL_U; break;
        case SCP_FIELD_Z: plane = PL_Z; break;
        case SCP_FIELD_LAM: plane = PL_LAM; break;
        case SCP_FIELD_MU: plane = PL_MU; break;
        case SCP_FIELD_DDYN: plane = PL_DD; break;
        case SCP_FIELD_COPY: plane = PL_CP; break;
        case SCP_FIELD_DUAL: plane = PL_DU; break;
        case SCP_FIELD_A: plane = PL_AR; mode = 1; break;
        case SCP_FIELD_B: plane = PL_B; mode = 2; break;
        case SCP_FIELD_D: plane = PL_D; break;
        case SCP_FIELD_BOXLO: plane = PL_LO; mode = 3; break;
        case SCP_FIELD_BOXHI: plane = PL_HI; mode = 3; break;
        case SCP_FIELD_HS: plane = PL_HS; break;
    }
    hipError_t e = p->prec == SCP_F32
                       ? launch_gather<float>(p->df, plane, w, mode, reinterpret_cast<float*>(dst_dev), p->stream)
                       : launch_gather<double>(p->dd, plane, w, mode, reinterpret_cast<double*>(dst_dev), p->stream);
    return hip_check(p, e, "gather launch");
}

size_t scp_problem_state_bytes(const scp_problem* p) {
    return p ? sizeof(StateHeader) + p->L.total : 0;
}

scp_status scp_problem_export_state(scp_problem* p, void* host, size_t bytes) {
    if (!p) return SCP_ERR_ARG;
    if (!host || bytes < scp_problem_state_bytes(p)) return fail(p, SCP_ERR_ARG, "export_state: buffer NULL or too small");
    TraceRange tr("scp_problem_export_state");
    StateHeader h{};
    h.magic = STATE_MAGIC;
    h.fingerprint = layout_fingerprint(p);
    h.arena_bytes = p->L.total;
    h.linearized = p->linearized ? 1 : 0;
    h.prec = (int32_t)p->prec;
    for (int k = 0; k < 3; ++k) h.lin_rho[k] = p->lin_rho[k];
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(static_cast<char*>(host) + sizeof h, p->arena, p->L.total, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_check(p, e, "export_state copy");
    std::memcpy(host, &h, sizeof h);
    return SCP_OK;
}

scp_status scp_problem_import_state(scp_problem* p, const void* host, size_t bytes) {
    if (!p) return SCP_ERR_ARG;
    if (!host || bytes != scp_problem_state_bytes(p)) return fail(p, SCP_ERR_ARG, "import_state: buffer NULL or of another size");
    StateHeader h;
    std::memcpy(&h, host, sizeof h);
    if (h.magic != STATE_MAGIC || h.arena_bytes != p->L.total || h.prec != (int32_t)p->prec ||
        h.fingerprint != layout_fingerprint(p))
        return fail(p, SCP_ERR_ARG, "import_state: not a state of a problem with this layout");
    TraceRange tr("scp_problem_import_state");
    hipError_t e = hipMemcpyAsync(p->arena, static_cast<const char*>(host) + sizeof h, p->L.total, hipMemcpyHostToDevice,
                                  p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_check(p, e, "import_state copy");
    p->linearized = h.linearized != 0;
    for (int k = 0; k < 3; ++k) p->lin_rho[k] = h.lin_rho[k];
    return SCP_OK;
}

scp_status scp_get_result(const scp_problem* cp, void* x_dev, void* u_dev, void* info_dev) {
    scp_problem* p = const_cast<scp_problem*>(cp);
    if (!p) return SCP_ERR_ARG;
    scp_status st = SCP_OK;
    if (x_dev) st = scp_get_field(p, SCP_FIELD_XBAR, x_dev);
    if (st == SCP_OK && u_dev) st = scp_get_field(p, SCP_FIELD_UBAR, u_dev);
    if (st == SCP_OK && info_dev) {
        hipError_t e = hipMemcpyAsync(info_dev, p->arena + p->L.o_info, (size_t)p->L.n_traj * SCP_INFO_FIELDS * 8,
                                      hipMemcpyDeviceToDevice, p->stream);
        st = hip_check(p, e, "info copy");
    }
    return st;
}

int64_t scp_problem_nodes(const scp_problem* p) { return p ? p->L.n_nodes : 0; }

int64_t scp_traj_node_offset(const scp_problem* p, int32_t t) {
    if (!p || t < 0 || t >= p->L.n_traj) return -1;
    return p->L.traj[(size_t)t * TR_FIELDS + TR_OFF];
}

scp_status scp_plan(const scp_problem_desc* desc, int32_t plan[5], int32_t* lane_table, size_t lane_cap) {
    g_create_error.clear();
    if (!plan) {
        g_create_error = "plan is NULL";
        return SCP_ERR_ARG;
    }
    Layout L;
    std::string err;
    if (!build_layout(desc, L, err)) {
        g_create_error = err;
        return SCP_ERR_ARG;
    }
    const size_t lanes = (size_t)L.n_wg * L.block;
    int cross = 0;
    for (int w = 0; w < L.n_wg; ++w) cross += (L.lane[lanes + w] & WG_CROSS) ? 1 : 0;
    plan[0] = L.persistent_ok ? L.block : 0;
    plan[1] = L.n_wg;
    plan[2] = cross;
    plan[3] = L.persistent_ok ? (int32_t)((long long)lanes - L.n_nodes) : 0;
    plan[4] = L.n_gslots;
    if (lane_table && L.persistent_ok && lane_cap >= lanes) std::memcpy(lane_table, L.lane.data(), lanes * sizeof(int32_t));
    return SCP_OK;
}

size_t scp_autotune_device_bytes(const scp_problem_desc* desc) {
    if (!desc) return 0;
    size_t best = 0;
    for (int b : {64, 128, 256})
        for (int pk : {SCP_PACK_ALIGNED, SCP_PACK_DENSE}) {
            scp_problem_desc d = *desc;
            d.block = b;
            d.pack = pk;
            Layout L;
            std::string err;
            if (!build_layout(&d, L, err)) return 0;
            best = std::max(best, L.total);
        }
    return best;
}

scp_status scp_autotune(const scp_problem_desc* desc, const scp_params* prm, const int32_t* cadences, int32_t n_cad,
                        int32_t reps, void* arena_dev, size_t arena_bytes, void* hip_stream, scp_tune_entry* table,
                        int32_t table_cap, int32_t* n_out, scp_tune_entry* best) {
    g_create_error.clear();
    auto bad = [](const std::string& m, scp_status st = SCP_ERR_ARG) {
        g_create_error = m;
        return st;
    };
    if (!desc || !prm || !n_out || !best) return bad("NULL argument");
    if (reps < 1) return bad("reps must be >= 1");
    if (n_cad < 0 || (n_cad > 0 && !cadences)) return bad("invalid cadence list");
    std::string err;
    if (!admm_valid(&prm->admm, err)) return bad(err);
    if (prm->scp_iters < 0) return bad("scp_iters must be >= 0");
    {
        Layout L;
        if (!build_layout(desc, L, err)) return bad(err);
    }
    std::vector<int> cads(cadences, cadences + n_cad);
    if (cads.empty()) cads.push_back(prm->admm.check_every);
    for (int c : cads)
        if (c < 0) return bad("cadences must be >= 0");
    *n_out = 0;
    const std::string key = tune_key(desc, prm, cads);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = it->second;
            return SCP_OK;
        }
    }
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipError_t e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    scp_status st = SCP_OK;
    int count = 0;
    bool found = false;
    scp_tune_entry b{};
    // one candidate: `reps` timed fresh solves after an untimed one
    auto time_one = [&](scp_problem* p, const scp_params& q, scp_tune_entry& en) {
        st = scp_reset(p);
        if (st == SCP_OK) st = scp_solve(p, &q);
        if (st == SCP_OK) e = hipEventRecord(ev0, stream);
        for (int r = 0; r < reps && st == SCP_OK && e == hipSuccess; ++r) {
            st = scp_reset(p);
            if (st == SCP_OK) st = scp_solve(p, &q);
        }
        if (st == SCP_OK && e == hipSuccess) e = hipEventRecord(ev1, stream);
        if (st == SCP_OK && e == hipSuccess) e = hipEventSynchronize(ev1);
        float ms = 0.f;
        if (st == SCP_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
        if (st != SCP_OK) g_create_error = p->err;
        if (st != SCP_OK || e != hipSuccess) return false;
        en.valid = 1;
        en.ms = (double)ms / reps;
        if (!found || en.ms < b.ms) {
            b = en;
            found = true;
        }
        return true;
    };
    // one lane per node: workgroup size x packing x cadence
    for (int blk : {64, 128, 256}) {
        for (int pk : {SCP_PACK_ALIGNED, SCP_PACK_DENSE}) {
            if (e != hipSuccess || st != SCP_OK) break;
            if (blk == 64 && pk == SCP_PACK_DENSE) continue;  // one wavefront: both packings coincide
            scp_problem_desc d = *desc;
            d.block = blk;
            d.pack = pk;
            Layout L;
            const bool fits = build_layout(&d, L, err) && L.persistent_ok && L.total <= arena_bytes;
            scp_problem* p = nullptr;
            if (fits) {
                st = scp_problem_create(&d, arena_dev, arena_bytes, hip_stream, &p);
                if (st != SCP_OK) break;
                if (p->L.n_gslots > 0 && p->L.n_wg > p->span_cap) {   // spanning groups not all resident
                    scp_problem_destroy(p);
                    p = nullptr;
                }
            }
            for (int c : cads) {
                scp_tune_entry en{blk, pk, c, 0, 0.0, 1};
                if (p) {
                    scp_params q = *prm;
                    q.form = SCP_FORM_PERSISTENT;
                    q.graph = 0;
                    q.lanes_per_node = 1;
                    q.admm.check_every = c;
                    if (!time_one(p, q, en)) break;
                }
                if (table && count < table_cap) table[count] = en;
                ++count;
            }
            scp_problem_destroy(p);
        }
    }
    // lane groups of four (one workgroup per trajectory): fixed ADMM budgets only
    if (e == hipSuccess && st == SCP_OK) {
        Layout L;
        const bool ok = build_layout(desc, L, err) && L.lanes4_ok && L.total <= arena_bytes;
        scp_problem* p = nullptr;
        if (ok) st = scp_problem_create(desc, arena_dev, arena_bytes, hip_stream, &p);
        for (int c : cads) {
            if (st != SCP_OK || e != hipSuccess) break;
            scp_tune_entry en{ok ? L.resident_block : 0, SCP_PACK_ALIGNED, c, 0, 0.0, 4};
            if (p && c == 0) {
                scp_params q = *prm;
                q.form = SCP_FORM_PERSISTENT;
                q.graph = 0;
                q.lanes_per_node = 4;
                q.admm.check_every = 0;
                if (!time_one(p, q, en)) break;
            }
            if (table && count < table_cap) table[count] = en;
            ++count;
        }
        scp_problem_destroy(p);
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    *n_out = count;
    if (st != SCP_OK) return st;
    if (e != hipSuccess) return bad(std::string("autotune timing: ") + hipGetErrorString(e), SCP_ERR_HIP);
    if (!found) return bad("no candidate workgroup size holds the longest trajectory or group", SCP_ERR_UNSUPPORTED);
    *best = b;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = b;
    return SCP_OK;
}

const char* scp_last_error(const scp_problem* p) {
    if (!p) return g_create_error.c_str();
    return p->err.c_str();
}

}  // extern "C"
