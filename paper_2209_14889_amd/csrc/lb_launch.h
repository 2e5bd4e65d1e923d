// Host-callable launch wrappers of the liblb kernels (defined in lb_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "lb_common.h"

namespace lbk {

// message returned by lb_last_error() on this thread
void set_last_error(const char *msg);

hipError_t launch_ib(bool advance, int nbodies, int ntiles, hipStream_t st, const SimDev *sims, BodyDev *bodies,
                     const int2 *blk, int cur, const int *d_t, int *d_status);
// walls: the variant with wall handling (needed when any simulation of the launch has walls);
// pol: the variant with the polarization field (needed unless P is zero in every simulation);
// cus: the device's compute units (work-groups of the first round are dealt to them in turn)
hipError_t launch_fused(int T, bool fp16, bool walls, bool pol, int grid, hipStream_t st, const SimDev *sims,
                        const BodyDev *bodies, const WorkItem *items, int n_items, int cur, int *d_t, int cus);
// resident fused work-groups per compute unit for work-group size T
int fused_blocks_per_cu(int T, bool fp16, bool walls, bool pol);
hipError_t launch_multipass(bool fp16, int nblocks, hipStream_t st, const SimDev *sims, const BodyDev *bodies,
                            const SiteBlock *blk, int cur, int *d_t);
hipError_t launch_readout(bool fp16, int nblocks, int block0, hipStream_t st, const SimDev *sims,
                          const BodyDev *bodies, const SiteBlock *blk, int cur, float *out);
hipError_t launch_sums(bool fp16, int sim, int nblocks, hipStream_t st, const SimDev *sims, int cur, double *partial,
                       double *out, double check_mass, int *d_status);
// body observables of bodies body0 .. body0+nbodies-1, 6 doubles each into out
hipError_t launch_body_force(hipStream_t st, const SimDev *sims, const BodyDev *bodies, int body0, int nbodies, int cur,
                             double *out);
// streaming device-to-device copy (bytes a multiple of 16, 16-byte aligned pointers)
hipError_t launch_stream_copy(hipStream_t st, const void *src, void *dst, size_t bytes);
hipError_t launch_pack(bool fp16, hipStream_t st, const float *src, void *dst, size_t n, float scale);

}  // namespace lbk
