// sun_internal.hpp -- launchers of the SU(N) kernels (N = 2, 4) and of the
// N-aware final quality reduction.
#pragma once

#include <hip/hip_runtime.h>

#include "gf_internal.hpp"

namespace gf {

hipError_t launch_sun_half_sweep(int prec, int nc, const Schedule &s, const CfgDesc *d_desc,
                                 const int *d_tile_cfg, const int *d_active, int ntiles, int parity,
                                 int reunit, hipStream_t st);
hipError_t launch_sun_pack(int prec, int nc, const Geom &g, const void *aos, void *U, int to_aos,
                           hipStream_t st);
hipError_t launch_sun_reunit(int prec, int nc, const Geom &g, void *U, hipStream_t st);
hipError_t launch_sun_quality(int prec, int nc, const CfgDesc *d_desc, const int *d_qtile_cfg,
                              const int *d_active, int nqtiles, double *d_partials, const SlabOrder &so,
                              hipStream_t st);
// k_quality_final with F and theta normalised for nc colours.
hipError_t launch_quality_final_nc(int nc, const CfgDesc *d_desc, int n, const double *d_partials,
                                   double *d_result, int *d_active, int *d_iters, int swept, double eps,
                                   int update_active, hipStream_t st);

}  // namespace gf
