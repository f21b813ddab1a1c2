// lbm_inst.hip -- the launchers (and so the kernels) of one storage mode and
// one kernel family, explicitly instantiated.  The build compiles this file
// once per pair, selected by
//   LBM_INST_ST      lbm_storage: 0 FP64, 1 FP32-shifted, 2 FP16-shifted,
//                    3 FP16 with a per-cell reference;
//   LBM_INST_FAMILY  1: single-step sweeps (step, moments, diagnostics),
//                    batched single steps, initialisation and the
//                    population permutation; 2: the two-step pass, alone
//                    and batched.
#include "lbm_kernels.hpp"

#if !defined(LBM_INST_ST) || !defined(LBM_INST_FAMILY)
#error "compile with -DLBM_INST_ST=<0..3> -DLBM_INST_FAMILY=<1|2>"
#endif

namespace lbmk {
#if LBM_INST_FAMILY == 1
LBM_DECLARE_FAMILY1(, LBM_INST_ST)
#else
LBM_DECLARE_FAMILY2(, LBM_INST_ST)
#endif
}  // namespace lbmk
