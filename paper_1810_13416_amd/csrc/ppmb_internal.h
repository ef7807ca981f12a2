// ppmb_internal.h -- declarations shared by the translation units of the
// HIP library (kernels, launchers and the C-ABI runtime).
#pragma once
#include <hip/hip_runtime.h>

#include "ppmb_dev.h"

namespace ppmb {

// fused 1-D pass over every pencil of the grid along `axis`
template <typename T>
hipError_t launch_sweep(const Geom &g, int axis, const T *in, T *out, const T *rho0, const T *p0,
                        const double *dtp, unsigned long long *counters, int heat, hipStream_t st);

// hydrostatic base state: FP64 RK4 node table (one thread), then cell values
hipError_t launch_base_state(const Geom &g, int kind, const double *params, double *table,
                             long table_len, double *rho0, double *p0, hipStream_t st);

// conversions between FP64 primitive perturbations and the stored conserved
// fields of the working precision
template <typename T>
hipError_t launch_prim_to_cons(const Geom &g, const double *const *prim, const double *rho0,
                               T *state, hipStream_t st);
template <typename T>
hipError_t launch_cons_to_prim(const Geom &g, const T *state, const double *rho0, double *prim,
                               hipStream_t st);
template <typename T>
hipError_t launch_widen(const T *src, double *dst, long count, hipStream_t st);
template <typename T>
hipError_t launch_narrow(const double *src, T *dst, long count, hipStream_t st);

// CFL reduction: smax (uint64 image of the FP64 maximum) and a flag word,
// then dt = cfl * dx / smax into *dtp
template <typename T>
hipError_t launch_cfl(const Geom &g, const T *state, const double *rho0, const double *p0,
                      unsigned long long *work, double cfl, double *dtp, hipStream_t st);

// conserved totals with a fixed reduction tree; out[8] on the device
template <typename T>
hipError_t launch_totals(const Geom &g, const T *state, const double *rho0, const double *p0,
                         double *partials, double *out, hipStream_t st);
constexpr int kTotalsBlocks = 1024;

hipError_t launch_set_scalar(double *dst, double v, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long *dst, int count, hipStream_t st);

}  // namespace ppmb
