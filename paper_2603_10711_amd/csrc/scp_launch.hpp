// Host-side launchers of the kernels (defined next to the kernels, called by the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "scp_layout.hpp"

namespace scp {

enum class PlainOp { Lin, Step1, Step234, Resid, Accept, Metrics, Reset, ResetState };

// models: bit 0 quadrotor present, bit 1 powered descent present; kmax: largest obstacle count.
template <class T>
hipError_t launch_plain(PlainOp op, const Dev<T>& dv, const KParams<T>& kp, int models, int kmax, int check, int j,
                        hipStream_t s);

template <class T>
hipError_t launch_gather(const Dev<T>& dv, int plane, int width, int mode, T* out, hipStream_t s);

// Persistent form: one workgroup per entry of the lane table, n_wg workgroups of `block`
// lanes.  Runs kp.n_scp SCP iterations.
template <class T>
hipError_t launch_persistent(const Dev<T>& dv, const KParams<T>& kp, int n_wg, int block, int models, int kmax,
                             hipStream_t s);

// ADMM iterations of a batch of one 6-DOF model (models: 4 quadrotor, 8 lander) resident in one
// workgroup per trajectory (`block` = 4 (N_max + 1) lanes rounded up to 64, at most 256):
// kp.max_iters iterations, fixed budget; the last one leaves the residual pieces that the Resid
// op completes.
template <class T>
hipError_t launch_resident(const Dev<T>& dv, const KParams<T>& kp, int n_traj, int block, int models, int kmax,
                           hipStream_t s);

// Static LDS of one persistent workgroup of `block` lanes (element size esz) for quadrotor
// launches with up to 8 obstacles, the largest workgroup state; 0 for an unsupported size.
size_t persistent_shared_bytes(int esz, int block);

// Server: scatter n staged admissions (records at blob + rec_off) into the pool, with cold
// initialization or in-place warm start; gather n finished requests into the output staging.
template <class T>
hipError_t launch_admit(const Dev<T>& dv, int block, const unsigned char* blob, int rec_off, int n, hipStream_t s);
template <class T>
hipError_t launch_collect(const Dev<T>& dv, const CollectRec* recs, int n, unsigned char* out, hipStream_t s);

}  // namespace scp
