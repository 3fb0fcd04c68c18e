// inst_weak.hip -- weak coupling (all M species lattices stored): double storage
// and arithmetic with a double record, and float storage with double arithmetic
// and a float record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp64_weak(int M, int walls, kern::Ops& o) { return kern::pick_m_any<double, double, double, true, false>(M, walls, o); }
bool pick_fp32_fp64_weak(int M, int walls, kern::Ops& o)
{
  return kern::pick_m_any<float, double, float, true, false>(M, walls, o);
}
}  // namespace mclbm
