// inst_fp32_fp64.hip -- kernels with float storage and double arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp32_fp64_weak(int M, int walls, kern::Ops& o);   // inst_weak.hip

bool pick_fp32_fp64(int M, int walls, int weak, kern::Ops& o)
{
  return weak ? pick_fp32_fp64_weak(M, walls, o) : kern::pick_m<float, double, float, false>(M, walls, o);
}
}  // namespace mclbm
