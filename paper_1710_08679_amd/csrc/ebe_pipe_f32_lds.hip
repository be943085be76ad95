// Pipelined and coloured EBE product forms: FP32, element geometry in LDS, the cases
// in one pass (the kernels are in pipe_kernel.h; the dtype / variant
// combinations compile in parallel).
#include "pipe_kernel.h"

namespace ebe {

#define EBE_INST(n)                                                                                     \
  template hipError_t launch_pipe<float, n, 2, true, 1>(const ebe_mesh*, const void*, void*, bool, bool, bool, \
                                                  const int*, hipStream_t, double*, bool);              \
  template hipError_t launch_pipe<float, n, 1, true, 1>(const ebe_mesh*, const void*, void*, bool, bool, bool, \
                                                  const int*, hipStream_t, double*, bool);
EBE_INST(1) EBE_INST(2) EBE_INST(3) EBE_INST(4) EBE_INST(5) EBE_INST(6) EBE_INST(7) EBE_INST(8)
EBE_INST(9) EBE_INST(10) EBE_INST(11) EBE_INST(12) EBE_INST(13) EBE_INST(14) EBE_INST(15) EBE_INST(16)
#undef EBE_INST

}  // namespace ebe
