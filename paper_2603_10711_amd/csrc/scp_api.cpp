// Host side of the C ABI declared in include/scp.h: validation, arena layout, packing of
// trajectories into persistent-kernel workgroups, upload, and the launch sequences of the
// plain and persistent forms.
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

using namespace scp;

namespace {

thread_local std::string g_create_error;

bool valid_model(int m) {
    return m == SCP_MODEL_QUAD_PM || m == SCP_MODEL_MARS3DOF || m == SCP_MODEL_QUAD_6DOF || m == SCP_MODEL_LANDER6;
}
bool quad_like(int m) { return m == SCP_MODEL_QUAD_PM || m == SCP_MODEL_QUAD_6DOF; }
// model bit of Layout::models
int model_bit(int m) {
    return m == SCP_MODEL_QUAD_PM ? 1 : m == SCP_MODEL_MARS3DOF ? 2 : m == SCP_MODEL_QUAD_6DOF ? 4 : 8;
}
const char* const kNoPersistent =
    "the persistent form needs trajectories of at most 256 nodes, consensus groups of at most 64 members and the "
    "point-mass quadrotor or 3-DOF powered-descent model, or a batch of one 6-DOF model alone with at most 64 "
    "nodes per trajectory and no consensus groups (resident ADMM); use the plain form";

// Pack units (single trajectories or whole consensus groups) of one model into workgroups of
// `block` lanes, first-fit decreasing by size.  Returns false if a unit does not fit.
struct Unit {
    int first_traj, n_traj, lanes, model;
};

struct Packed {
    std::vector<int> lane;      // n_wg * block node indices, -1 idle
    std::vector<int> wg_info;   // n_wg: model | WG_CROSS | WG_SPAN
    std::vector<int> wg_group;  // 2 * n_wg: spanning group slot, workgroups of that group
    int n_wg = 0;
    int n_gslots = 0;
};

// Aligned packing: a unit of at most 64 lanes never straddles a wavefront boundary and a longer
// unit starts on one.  Dense packing: first fit over the whole workgroup.  A workgroup in which
// no unit straddles a wavefront boundary exchanges neighbour values with wavefront shifts; the
// others (WG_CROSS) exchange them through LDS.  A consensus group larger than one workgroup is
// split by member over workgroups of its own (WG_SPAN), each member whole in one workgroup.
bool pack(const std::vector<Unit>& units, const std::vector<int>& traj_off, const std::vector<int>& horizon,
          int block, bool aligned, Packed& out) {
    constexpr int W = 64;
    const int nw = aligned ? block / W : 1;   // fill slots per workgroup
    const int cap = aligned ? W : block;      // lanes per fill slot
    out = Packed{};
    struct Wg {
        std::vector<int> fill;
        int index;
    };
    auto new_wg = [&](std::vector<Wg>& set, int model, int extra) {
        set.push_back(Wg{std::vector<int>(nw, 0), out.n_wg++});
        out.lane.resize((size_t)out.n_wg * block, -1);
        out.wg_info.push_back(model | extra);
        out.wg_group.push_back(0);
        out.wg_group.push_back(0);
        return (int)set.size() - 1;
    };
    // first free position for `lanes` lanes in workgroup q of `set`; returns the fill slot or -1
    auto find_slot = [&](const Wg& g, int lanes) {
        if (lanes <= cap) {
            for (int v = 0; v < nw; ++v)
                if (g.fill[v] + lanes <= cap) return v;
            return -1;
        }
        const int k = (lanes + cap - 1) / cap;  // fill slots spanned, all empty
        for (int v = 0; v + k <= nw; ++v) {
            bool empty = true;
            for (int e = v; e < v + k; ++e) empty = empty && g.fill[e] == 0;
            if (empty) return v;
        }
        return -1;
    };
    auto place = [&](Wg& g, int v, int first_traj, int n_traj, int lanes) {
        const int off = v * cap + g.fill[v];  // lane offset inside the workgroup
        if (off / W != (off + lanes - 1) / W) out.wg_info[g.index] |= WG_CROSS;
        int base = g.index * block + off;
        for (int t = first_traj; t < first_traj + n_traj; ++t)
            for (int i = 0; i <= horizon[t]; ++i) out.lane[base++] = traj_off[t] + i;
        int rest = lanes;
        for (int e = v; rest > 0; ++e) {
            const int take = std::min(rest, cap - g.fill[e]);
            g.fill[e] += take;
            rest -= take;
        }
    };
    for (int model : {SCP_MODEL_QUAD_PM, SCP_MODEL_MARS3DOF}) {
        std::vector<int> idx;
        for (int u = 0; u < (int)units.size(); ++u)
            if (units[u].model == model) idx.push_back(u);
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return units[a].lanes > units[b].lanes; });
        std::vector<Wg> shared;  // this model's workgroups open to any unit
        for (int u : idx) {
            const Unit& un = units[u];
            if (un.lanes <= block) {
                int q = -1, v = -1;
                for (int c = 0; c < (int)shared.size() && q < 0; ++c) {
                    v = find_slot(shared[c], un.lanes);
                    if (v >= 0) q = c;
                }
                if (q < 0) {
                    q = new_wg(shared, model, 0);
                    v = find_slot(shared[q], un.lanes);
                }
                place(shared[q], v, un.first_traj, un.n_traj, un.lanes);
                continue;
            }
            // spanning consensus group: members over workgroups of its own
            const int L = horizon[un.first_traj] + 1;
            if (un.n_traj < 2 || L > block || un.n_traj > GX_MEMBERS) return false;
            std::vector<Wg> own;
            const int slot = out.n_gslots++;
            for (int m = 0; m < un.n_traj; ++m) {
                int q = (int)own.size() - 1, v = q >= 0 ? find_slot(own[q], L) : -1;
                if (v < 0) {
                    q = new_wg(own, model, WG_SPAN);
                    v = find_slot(own[q], L);
                }
                place(own[q], v, un.first_traj + m, 1, L);
            }
            if ((int)own.size() > GX_MAX_WG) return false;
            for (const Wg& g : own) {
                out.wg_group[2 * g.index] = slot;
                out.wg_group[2 * g.index + 1] = (int)own.size();
            }
        }
    }
    return true;
}

}  // namespace

namespace scp {

bool build_layout(const scp_problem_desc* d, Layout& L, std::string& err) {
    if (!d) { err = "desc is NULL"; return false; }
    if (d->n_traj < 1) { err = "n_traj must be >= 1"; return false; }
    if (d->prec != SCP_F32 && d->prec != SCP_F64) { err = "invalid precision"; return false; }
    if (!d->model || !d->horizon || !d->params || !d->x_guess || !d->u_guess) { err = "NULL array in desc"; return false; }
    if (d->block != 0 && d->block != 64 && d->block != 128 && d->block != 256) { err = "block must be 0, 64, 128 or 256"; return false; }
    if (d->pack != SCP_PACK_ALIGNED && d->pack != SCP_PACK_DENSE) { err = "pack must be SCP_PACK_ALIGNED or SCP_PACK_DENSE"; return false; }
    L.n_traj = d->n_traj;
    L.esz = d->prec == SCP_F32 ? 4 : 8;
    L.traj.assign((size_t)L.n_traj * TR_FIELDS, 0);
    std::vector<int> traj_off(L.n_traj), horizon(L.n_traj);
    long long off = 0;
    for (int t = 0; t < L.n_traj; ++t) {
        const int m = d->model[t], N = d->horizon[t];
        if (!valid_model(m)) { err = "invalid model id at trajectory " + std::to_string(t); return false; }
        if (N < 1 || N > SCP_MAX_N) { err = "horizon out of range at trajectory " + std::to_string(t); return false; }
        const double* prm = d->params + (size_t)t * SCP_PARAM_STRIDE;
        const double K = prm[SCP_P_NOBS];
        if (quad_like(m) && !(K >= 0 && K <= SCP_MAX_OBS && K == std::floor(K))) {
            err = "obstacle count out of range at trajectory " + std::to_string(t);
            return false;
        }
        if (!(prm[SCP_P_H] > 0) || !std::isfinite(prm[SCP_P_H])) { err = "step size must be positive"; return false; }
        if (!(prm[SCP_P_DELTA] > 0)) { err = "trust radius must be positive"; return false; }
        int* r = &L.traj[(size_t)t * TR_FIELDS];
        r[TR_MODEL] = m;
        r[TR_N] = N;
        r[TR_OFF] = (int)off;
        r[TR_K] = quad_like(m) ? (int)K : 0;
        r[TR_BALL] = (m == SCP_MODEL_QUAD_PM && std::isfinite(prm[SCP_P_UBALL])) ? 1 : 0;
        r[TR_GFIRST] = t;
        r[TR_GSIZE] = 1;
        r[TR_MEMBER] = 0;
        traj_off[t] = (int)off;
        horizon[t] = N;
        off += N + 1;
        L.models |= model_bit(m);
        L.kmax = std::max(L.kmax, r[TR_K]);
        if (off > (1LL << 30)) { err = "too many nodes"; return false; }
    }
    L.n_nodes = (int)off;
    L.P = (int)((off + 255) / 256 * 256);
    // consensus groups
    std::vector<Unit> units;
    int t = 0;
    while (t < L.n_traj) {
        int e = t + 1;
        const int gid = d->group ? d->group[t] : -1;
        if (gid >= 0) {
            while (e < L.n_traj && d->group[e] == gid) ++e;
            for (int q = t; q < e; ++q) {
                if (d->model[q] != d->model[t] || d->horizon[q] != d->horizon[t]) {
                    err = "members of a consensus group must share model and horizon";
                    return false;
                }
            }
            if (e - t > 1 && d->model[t] == SCP_MODEL_LANDER6) {
                err = "consensus groups of the 6-DOF lander are not supported";
                return false;
            }
            for (int q = e; q < L.n_traj; ++q)
                if (d->group[q] == gid) {
                    err = "members of a consensus group must be consecutive";
                    return false;
                }
        }
        for (int q = t; q < e; ++q) {
            int* r = &L.traj[(size_t)q * TR_FIELDS];
            r[TR_GFIRST] = t;
            r[TR_GSIZE] = e - t;
            r[TR_MEMBER] = q - t;
        }
        if (e - t > 1) L.groups.push_back(t);
        units.push_back({t, e - t, (e - t) * (horizon[t] + 1), d->model[t]});
        t = e;
    }
    L.n_groups = (int)L.groups.size();
    L.node_traj.assign(L.P, -1);
    for (int q = 0; q < L.n_traj; ++q)
        for (int i = 0; i <= horizon[q]; ++i) L.node_traj[traj_off[q] + i] = q;
    // persistent-kernel packing: the requested block, or the candidate with the lowest cost
    // estimate.  The kernel runs one wave per SIMD (1024 SIMDs on the chip); waves of one
    // workgroup wait for each other at every exchange barrier, so at equal wave rounds a
    // smaller workgroup wins, and the idle-lane count breaks ties.
    std::vector<int> cands = d->block ? std::vector<int>{d->block} : std::vector<int>{64, 128, 256};
    if (d->prec == SCP_F64) cands.erase(std::remove(cands.begin(), cands.end(), 256), cands.end());
    long best_idle = -1;
    double best_score = 0.0;
    if (L.models & (4 | 8)) cands.clear();  // the 6-DOF models run in the plain form only
    for (int b : cands) {
        Packed pk;
        if (!pack(units, traj_off, horizon, b, d->pack == SCP_PACK_ALIGNED, pk)) continue;
        const long idle = (long)pk.n_wg * b - L.n_nodes;
        const double waves = (double)pk.n_wg * (b / 64);
        // spanning groups pay a group barrier per ADMM iteration: fewer workgroups per group win
        const double score = std::ceil(waves / 1024.0) * (1.0 + 0.05 * (b / 64 - 1)) + (pk.n_gslots ? 64.0 / b : 0.0);
        if (best_idle < 0 || score < best_score || (score == best_score && idle < best_idle)) {
            best_idle = idle;
            best_score = score;
            L.block = b;
            L.n_wg = pk.n_wg;
            L.n_gslots = pk.n_gslots;
            L.lane = pk.lane;
            L.lane.insert(L.lane.end(), pk.wg_info.begin(), pk.wg_info.end());
            L.lane.insert(L.lane.end(), pk.wg_group.begin(), pk.wg_group.end());
        }
    }
    L.persistent_ok = best_idle >= 0;
    if (!L.persistent_ok) {
        L.block = 0;
        L.n_wg = 0;
        L.n_gslots = 0;
        L.lane.assign(1, -1);
    }
    // a batch of one 6-DOF model alone, without consensus groups: ADMM resident in one workgroup
    // per trajectory, four lanes per node
    int max_nodes = 0;
    for (int q = 0; q < L.n_traj; ++q) max_nodes = std::max(max_nodes, horizon[q] + 1);
    L.resident_ok = (L.models == 4 || L.models == 8) && L.n_groups == 0 && max_nodes <= RESIDENT_MAX_NODES;
    // the point-mass models in lane groups of four: the same resident ADMM
    L.lanes4_ok = (L.models & ~3) == 0 && L.n_groups == 0 && max_nodes <= RESIDENT_MAX_NODES;
    L.resident_block = (L.resident_ok || L.lanes4_ok) ? (4 * max_nodes + 63) / 64 * 64 : 0;
    // arena
    size_t o = 0;
    L.o_traj = o; o = align_up(o + L.traj.size() * 4);
    L.o_node_traj = o; o = align_up(o + (size_t)L.P * 4);
    L.o_lane = o; o = align_up(o + L.lane.size() * 4);
    L.o_groups = o; o = align_up(o + std::max<size_t>(1, L.groups.size()) * 4);
    L.o_params = o; o = align_up(o + (size_t)L.n_traj * SCP_PARAM_STRIDE * L.esz);
    L.o_planes = o; o = align_up(o + (size_t)NPLANES * L.P * L.esz);
    L.o_rt = o; o = align_up(o + (size_t)L.n_traj * RT_FIELDS * L.esz);
    L.o_info = o; o = align_up(o + (size_t)L.n_traj * SCP_INFO_FIELDS * 8);
    L.o_flags = o; o = align_up(o + (size_t)L.n_traj * FL_FIELDS * 4);
    L.o_red = o; o = align_up(o + (size_t)L.n_traj * 2 * 8);
    L.o_gsync = o; o = align_up(o + (size_t)L.n_gslots * GX_SYNC_STRIDE * 4);
    L.o_gx = o; o = align_up(o + (size_t)L.n_gslots * 2 * GX_MEMBERS * GX_WIDTH * L.esz);
    L.total = o;
    return true;
}

template <class T>
Dev<T> make_dev(const Layout& L, char* base) {
    Dev<T> dv;
    dv.traj = reinterpret_cast<const int*>(base + L.o_traj);
    dv.node_traj = reinterpret_cast<const int*>(base + L.o_node_traj);
    dv.lane_node = reinterpret_cast<const int*>(base + L.o_lane);
    dv.params = reinterpret_cast<const T*>(base + L.o_params);
    dv.planes = reinterpret_cast<T*>(base + L.o_planes);
    dv.rt = reinterpret_cast<T*>(base + L.o_rt);
    dv.info = reinterpret_cast<double*>(base + L.o_info);
    dv.flags = reinterpret_cast<int*>(base + L.o_flags);
    dv.red = reinterpret_cast<unsigned long long*>(base + L.o_red);
    dv.n_traj = L.n_traj;
    dv.P = L.P;
    dv.n_nodes = L.n_nodes;
    dv.n_groups = L.n_groups;
    dv.groups = reinterpret_cast<const int*>(base + L.o_groups);
    const int* lanes = reinterpret_cast<const int*>(base + L.o_lane);
    dv.wg_list = nullptr;
    dv.wg_info = lanes + (size_t)L.n_wg * L.block;
    dv.wg_group = dv.wg_info + L.n_wg;
    dv.gsync = reinterpret_cast<unsigned*>(base + L.o_gsync);
    dv.gx = reinterpret_cast<T*>(base + L.o_gx);
    dv.n_gslots = L.n_gslots;
    return dv;
}

template Dev<float> make_dev<float>(const Layout&, char*);
template Dev<double> make_dev<double>(const Layout&, char*);

}  // namespace scp

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
           a.lanes_per_node == b.lanes_per_node;
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
    const Dev<T>& dv = *reinterpret_cast<const Dev<T>*>(p->prec == SCP_F32 ? (const void*)&p->df : (const void*)&p->dd);
    KParams<T> kp = kparams<T>(a, nullptr);
    hipError_t e = launch_plain<T>(PlainOp::Lin, dv, kp, p->L.models, p->L.kmax, 0, 0, p->stream);
    return hip_check(p, e, "linearize launch");
}

template <class T>
scp_status do_admm(scp_problem* p, const admm_params* a) {
    const Dev<T>& dv = *reinterpret_cast<const Dev<T>*>(p->prec == SCP_F32 ? (const void*)&p->df : (const void*)&p->dd);
    KParams<T> kp = kparams<T>(a, nullptr);
    return run_plain_admm<T>(p, dv, kp);
}

template <class T>
scp_status do_solve(scp_problem* p, const scp_params* s) {
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
        e = launch_persistent<T>(dv, kp, L.n_wg, L.block, L.models, L.kmax, p->stream);
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
