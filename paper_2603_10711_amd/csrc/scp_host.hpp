// Host-side planning shared by the problem API and the server: validation of a description,
// packing of trajectories into persistent-kernel workgroups, and the arena layout.
#pragma once

#include <string>
#include <vector>

#include "../../include/scp.h"
#include "scp_layout.hpp"

namespace scp {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int n_traj = 0, n_nodes = 0, P = 0;
    int models = 0, kmax = 0;
    int block = 0, n_wg = 0;
    bool persistent_ok = false;
    // 6-DOF quadrotor batches: ADMM resident in one workgroup per trajectory of resident_block
    // lanes (four per node)
    bool resident_ok = false;
    int resident_block = 0;
    // point-mass quadrotor / powered descent batches in lane groups of four (lanes_per_node = 4):
    // at most RESIDENT_MAX_NODES nodes per trajectory, no consensus groups; resident_block lanes
    bool lanes4_ok = false;
    int n_groups = 0;
    size_t esz = 4;
    // byte offsets inside the arena
    size_t o_traj, o_node_traj, o_lane, o_groups, o_params, o_planes, o_rt, o_info, o_flags, o_red, total;
    std::vector<int> traj;       // n_traj * TR_FIELDS
    std::vector<int> node_traj;  // P
    std::vector<int> lane;       // n_wg * block lanes, then wg_info [n_wg], then wg_group [2 n_wg]
    std::vector<int> groups;     // first trajectory of each multi-member group
    int n_gslots = 0;            // consensus groups spanning several workgroups
    size_t o_gsync = 0, o_gx = 0;
};

// Validate the description and lay out its arena (packing included).
bool build_layout(const scp_problem_desc* d, Layout& L, std::string& err);

// Longest wait at a spanning-group barrier in ticks of the device wall clock (100 MHz) for
// scp_params.group_wait_ms: 0 = 20 ms, < 0 = give up at the first wait.
inline unsigned long long group_wait_ticks(double ms) {
    if (ms < 0.0) return 0ull;
    if (ms == 0.0) ms = 20.0;
    const double t = ms * 1.0e5;
    return t >= 1.8e19 ? ~0ull : (unsigned long long)t;
}

// Workgroups of `block` lanes of the persistent kernel variant for consensus groups spanning
// several workgroups that the device keeps resident at once (occupancy of that kernel times the
// device's compute units); 0 if the query fails.  esz: element size (4 or 8).
int persistent_span_resident_cap(int esz, int block, int models, int kmax);

// No-allocation arena (scp_problem_create_noalloc): the error message of a failed create, the mark
// that makes scp_problem_destroy release the device's arena, and that release.
void set_create_error(const std::string& msg);
void problem_mark_noalloc(scp_problem* p, int dev);
void noalloc_release(int dev);

// Device views of an arena laid out by build_layout.
template <class T>
Dev<T> make_dev(const Layout& L, char* base);

}  // namespace scp
