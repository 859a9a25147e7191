// launch.hpp -- host-side launchers of the path kernels (one set per path
// precision and dynamics, defined in paths_<prec>_<dyn>.hip).
#pragma once

#include "bmotor.h"
#include "common.hpp"

namespace bm {

struct ScanArgs;

#define BM_DECLARE_LAUNCHERS(SUF)                                                                 \
    hipError_t launch_init_##SUF(int pot, int noise, const KArgs &a, hipStream_t s);               \
    hipError_t launch_advance_##SUF(int pot, int noise, int ppl, int block, const KArgs &a,       \
                                    hipStream_t s);                                                \
    hipError_t launch_scan_##SUF(int pot, int noise, int ppl, int block, int groups_per_cu,       \
                                 int n_cu, const ScanArgs &a, hipStream_t s);                       \
    hipError_t launch_advance_sc_##SUF(int pot, int block, const KArgs &a, hipStream_t s);

BM_DECLARE_LAUNCHERS(f32_od)
BM_DECLARE_LAUNCHERS(f32_in)
BM_DECLARE_LAUNCHERS(f64_od)
BM_DECLARE_LAUNCHERS(f64_in)
#undef BM_DECLARE_LAUNCHERS

// per-path velocity + wave partials, and the state export (depend on precision and L only)
hipError_t launch_velocity_f32(int pot, const KArgs &a, hipStream_t s);
hipError_t launch_velocity_f64(int pot, const KArgs &a, hipStream_t s);
hipError_t launch_density_f32(int pot, const KArgs &a, uint32_t n_bins, unsigned long long *hist, hipStream_t s);
hipError_t launch_density_f64(int pot, const KArgs &a, uint32_t n_bins, unsigned long long *hist, hipStream_t s);
// flags of the export: READ_VP the per-path velocity exists (steps done > window
// start), READ_SNAP the window snapshot exists (steps done >= window start)
constexpr int READ_VP = 1, READ_SNAP = 2;
hipError_t launch_read_f32(int pot, const KArgs &a, double *x, double *v, int64_t *nz, double *vp,
                           int flags, bm_path *st, hipStream_t s);
hipError_t launch_read_f64(int pot, const KArgs &a, double *x, double *v, int64_t *nz, double *vp,
                           int flags, bm_path *st, hipStream_t s);
hipError_t launch_write_f32(int pot, const KArgs &a, const bm_path *st, uint32_t snap, hipStream_t s);
hipError_t launch_write_f64(int pot, const KArgs &a, const bm_path *st, uint32_t snap, hipStream_t s);

} // namespace bm
