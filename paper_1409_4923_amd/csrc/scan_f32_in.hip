// Persistent scan kernels: float state, inertial dynamics.
#define BM_REAL float
#define BM_DYN 1
#define BM_SUF f32_in
#define BM_MAX_PPL 2
#include "scan_tu.inc"
