// Persistent scan kernels: double state, inertial dynamics.
#define BM_REAL double
#define BM_DYN 1
#define BM_SUF f64_in
#define BM_MAX_PPL 1
#include "scan_tu.inc"
