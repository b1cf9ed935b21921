// Host-side planning of a batch, shared by the problem API and the request server and free of
// device code: validation of a description, packing of trajectories (and whole consensus groups)
// into persistent-kernel workgroups, and the arena layout.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/scp.h"
#include "scp_host.hpp"
#include "scp_layout.hpp"

using namespace scp;

namespace {

bool valid_model(int m) {
    return m == SCP_MODEL_QUAD_PM || m == SCP_MODEL_MARS3DOF || m == SCP_MODEL_QUAD_6DOF || m == SCP_MODEL_LANDER6;
}
bool quad_like(int m) { return m == SCP_MODEL_QUAD_PM || m == SCP_MODEL_QUAD_6DOF; }
// model bit of Layout::models
int model_bit(int m) {
    return m == SCP_MODEL_QUAD_PM ? 1 : m == SCP_MODEL_MARS3DOF ? 2 : m == SCP_MODEL_QUAD_6DOF ? 4 : 8;
}

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
