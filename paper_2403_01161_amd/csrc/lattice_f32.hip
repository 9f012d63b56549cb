// Lattice kernels and launchers for SF32 population storage (one
// translation unit per storage type, compiled in parallel).
#include "lattice_kernels.h"

namespace ibmlb {
template hipError_t launch_lattice_c<SF32>(const Geom&, const LatticeParams&, const DevPtrs&, int, bool, const double*,
                                          int, int, hipStream_t, hipEvent_t, hipEvent_t, const MrtRates*,
                                          const ChiRates*);
template hipError_t launch_lattice_batch_c<SF32>(const LatDesc*, const int2*, const int*, const int*, const int*, int,
                                                long long, int, bool, hipStream_t);
}  // namespace ibmlb
