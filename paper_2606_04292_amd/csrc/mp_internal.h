// Launchers of the FP32 correction cycles (kernels_mp.hip).
#pragma once

#include "rs_internal.h"
#include "soil_mp.h"

namespace rs {

Law32 make_law32(const Law &L);
void launch_sweep32(const Geo &g, const Law32 &law, float a, const double *beta, float lambdaU,
                    const float *K, const float *rhs, const float *pb, float *dl, int nsweeps,
                    hipStream_t s);
void launch_residual32(const Geo &g, const Law32 &law, float a, const double *beta, const float *K,
                       const float *rhs, const float *pb, const float *dl, float *r, hipStream_t s);
void launch_coarse_rhs32(const Geo &g, const Law32 &law, float a, const double *beta,
                         const float *K, const float *pb, const float *dbar, float *rhs, float *dl,
                         hipStream_t s);
void launch_restrict32(const Geo &gc, const Geo &gf, const float *dl_f, const float *r_f,
                       float *dbar_c, float *rhs_c, hipStream_t s);
void launch_prolong32(const Geo &gf, const Geo &gc, const float *dl_c, const float *dbar_c,
                      float *dl_f, hipStream_t s);
// psi_b of levels 1 .. nlev-1 by injection from level 0, in one launch
// (geo[l] and pb[l]: level l's geometry and FP32 base state).
void launch_inject_base32(const Geo *geo, float *const *pb, int nlev, hipStream_t s);
void launch_to_f32(long long N, const double *src, float *dst, hipStream_t s);
void launch_apply_delta(long long N, const float *dl, double *psi64, hipStream_t s);
// The FP32 correction cycle from level top (all of whose levels hold at most
// kTailNodes nodes) down to level last and back, in one work-group.
void launch_vcycle_tail32(const TailArgs *args_dev, int top, int last, const Law32 &law, float a,
                          int nu1, int nu2, int nuc, int dim, hipStream_t s);

}  // namespace rs
