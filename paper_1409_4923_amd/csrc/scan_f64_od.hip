// Persistent scan kernels: double state, overdamped dynamics.
#define BM_REAL double
#define BM_DYN 0
#define BM_SUF f64_od
#define BM_MAX_PPL 1
#include "scan_tu.inc"
