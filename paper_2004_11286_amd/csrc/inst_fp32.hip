// inst_fp32.hip -- kernels with float storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
// open ends, free-slip walls, weak coupling and C_v(T) are compiled for FP64 arithmetic only
bool pick_fp32(int M, int walls, int weak, int cvt, kern::Ops& o)
{
  return !weak && !cvt && walls <= 1 && kern::pick_m<float, float, float, false>(M, walls, o);
}
}  // namespace mclbm
