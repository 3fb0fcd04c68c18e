// inst_weak_cvt.hip -- weak coupling with temperature-dependent specific heats
// and transport: double storage and arithmetic with a double record, and float
// storage with double arithmetic and a float record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp64_weak_cvt(int M, int walls, kern::Ops& o)
{
  return kern::pick_m_any<double, double, double, true, true>(M, walls, o);
}
bool pick_fp32_fp64_weak_cvt(int M, int walls, kern::Ops& o)
{
  return kern::pick_m_any<float, double, float, true, true>(M, walls, o);
}
}  // namespace mclbm
