// host.hpp -- host-side helpers shared by the ensemble and scan entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "bmotor.h"
#include "common.hpp"

namespace bm {
namespace host {

int fail(int code, const char *fmt, ...);           // set the thread's message, return code
int ok();                                           // clear the message, return BM_OK
int hip_fail(hipError_t e, const char *what);       // BM_ERR_DEVICE with HIP's message
const char *last_error_text();

int validate(const bm_model *m, const bm_run *r);   // argument checks of one (model, run)
double step_of(const bm_model *m, const bm_run *r); // dt
size_t table_entries(const bm_run *r);              // forcing table length (period + 16)
void forcing_table(const bm_model *m, const bm_run *r, std::vector<double> &tab);
PointConst point_const(const bm_model *m, const bm_run *r, const void *d_tab);
int check_device(int *dev_out);                     // a gfx950 device is current

// Launch shape used when the caller passes no bm_tune: set by bm_tune_set_default
// (or bm_scan_autotune), else paths_per_lane 1, block 256, groups_per_cu 0.
bm_tune default_tune(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec);
size_t queue_lds_bytes(uint32_t noise, uint32_t prec, uint32_t ppl, uint32_t block);
int check_tune(const bm_tune *t, uint32_t noise, uint32_t prec);

} // namespace host
} // namespace bm
