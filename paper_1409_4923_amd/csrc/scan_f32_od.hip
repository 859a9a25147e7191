// Persistent scan kernels: float state, overdamped dynamics.
#define BM_REAL float
#define BM_DYN 0
#define BM_SUF f32_od
#define BM_MAX_PPL 2
#include "scan_tu.inc"
