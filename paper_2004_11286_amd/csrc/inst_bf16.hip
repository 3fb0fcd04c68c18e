// inst_bf16.hip -- kernels with __bf16 storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
// open ends, free-slip walls, weak coupling and C_v(T) are compiled for FP64 arithmetic only
bool pick_bf16(int M, int walls, int weak, int cvt, kern::Ops& o)
{
  return !weak && !cvt && walls <= 1 && kern::pick_m<__bf16, float, float, false>(M, walls, o);
}
}  // namespace mclbm
