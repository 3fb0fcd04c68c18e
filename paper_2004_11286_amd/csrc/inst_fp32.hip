// inst_fp32.hip -- kernels with float storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
// weak coupling is compiled for FP64 arithmetic only
bool pick_fp32(int M, int walls, int weak, kern::Ops& o)
{
  return !weak && kern::pick_m<float, float, float, false>(M, walls, o);
}
}  // namespace mclbm
