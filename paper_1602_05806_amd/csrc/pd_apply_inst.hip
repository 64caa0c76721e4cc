// One (precision, degree) instantiation of the operator-apply kernels and their launchers:
// compiled once per pair with -DPD_INST_T=<double|float> -DPD_INST_N=<0..8> (see the Makefile),
// so the kernels of different degrees build in parallel.
#include "pd_apply_kernels.h"

#if !defined(PD_INST_T) || !defined(PD_INST_N)
#error "pd_apply_inst.hip needs PD_INST_T and PD_INST_N"
#endif

namespace pdk {
template hipError_t launch_apply_N<PD_INST_T, PD_INST_N>(const ApplyLaunch&, hipStream_t);
template unsigned blocks_N<PD_INST_T, PD_INST_N>(const ApplyLaunch&);
}  // namespace pdk
