// The fused phase-field step with 16-bit population storage (half and bfloat16 codes of
// g_i / w_i): the kernels of lbm_ch_step.hip instantiated for those storage modes only,
// in a translation unit of their own so that they can be built with machine-level
// loop-invariant code motion off (-mllvm -disable-machine-licm, see build.py).  With it
// on, the compiler keeps loop-invariant values of the unrolled march in registers,
// the 16-bit decode pushes the kernel past its 128-register budget, and it spills
// (5-6 registers); with it off it needs 115 and runs about 6 % faster at 2048^2.  The
// float32 kernels are faster with it on and stay in lbm_ch_step.hip.
#define LBM_STEP_16BIT_TU 1
#include "lbm_ch_step.hip"
