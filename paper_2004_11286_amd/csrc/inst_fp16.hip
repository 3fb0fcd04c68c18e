// inst_fp16.hip -- kernels with _Float16 storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
// weak coupling is compiled for FP64 arithmetic only
bool pick_fp16(int M, int walls, int weak, kern::Ops& o)
{
  return !weak && kern::pick_m<_Float16, float, float, false>(M, walls, o);
}
}  // namespace mclbm
