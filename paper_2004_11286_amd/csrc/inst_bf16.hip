// inst_bf16.hip -- kernels with __bf16 storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
// weak coupling is compiled for FP64 arithmetic only
bool pick_bf16(int M, int walls, int weak, kern::Ops& o)
{
  return !weak && kern::pick_m<__bf16, float, float, false>(M, walls, o);
}
}  // namespace mclbm
