// instances.hip -- explicit instantiations of the kernels for one storage type and one
// scheme, selected at compile time (-DMRL_T=double|float -DMRL_S=0..4). The build compiles
// this file once per pair, in parallel; mrlbm.hip only refers to the instances.
#include "mrlbm_kernels.h"

#ifndef MRL_T
#error "MRL_T (double or float) must be defined"
#endif
#ifndef MRL_S
#error "MRL_S (0..4) must be defined"
#endif

namespace mrl {
template __global__ void k_init<MRL_T, MRL_S>(const Desc*, State*, const double*, long long);
template __global__ void k_steps<MRL_T, MRL_S, 1>(const Desc*, State*, const int*, int, int, int, int);
template __global__ void k_steps<MRL_T, MRL_S, 2>(const Desc*, State*, const int*, int, int, int, int);
template __global__ void k_steps<MRL_T, MRL_S, 3>(const Desc*, State*, const int*, int, int, int, int);
template __global__ void k_query<MRL_T, MRL_S, 1>(const Desc*, State*, int, int, double*);
template __global__ void k_query<MRL_T, MRL_S, 2>(const Desc*, State*, int, int, double*);
template __global__ void k_query<MRL_T, MRL_S, 3>(const Desc*, State*, int, int, double*);
// variants for runs whose tree arrays live in device memory (J above the on-chip limit)
template __global__ void k_steps<MRL_T, MRL_S, 1, false, false, true>(const Desc*, State*, const int*, int, int, int, int);
template __global__ void k_steps<MRL_T, MRL_S, 2, false, false, true>(const Desc*, State*, const int*, int, int, int, int);
template __global__ void k_steps<MRL_T, MRL_S, 3, false, false, true>(const Desc*, State*, const int*, int, int, int, int);
template __global__ void k_query<MRL_T, MRL_S, 1, true>(const Desc*, State*, int, int, double*);
template __global__ void k_query<MRL_T, MRL_S, 2, true>(const Desc*, State*, int, int, double*);
template __global__ void k_query<MRL_T, MRL_S, 3, true>(const Desc*, State*, int, int, double*);
// variant that can run the reconstructed collision (gamma = 1)
template __global__ void k_steps<MRL_T, MRL_S, 1, false, true>(const Desc*, State*, const int*, int, int, int, int);
#if MRL_LRN
// variant that can run the refinement predictor (FP64 storage, gamma = 1)
template __global__ void k_steps<MRL_T, MRL_S, 1, true>(const Desc*, State*, const int*, int, int, int, int);
#endif
}  // namespace mrl
