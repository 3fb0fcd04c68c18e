// inst_fp32_fp64.hip -- kernels with float storage and double arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp32_fp64_weak(int M, int walls, kern::Ops& o);   // inst_weak.hip
bool pick_fp32_fp64_cvt(int M, int walls, kern::Ops& o);    // inst_cvt.hip
bool pick_fp32_fp64_weak_cvt(int M, int walls, kern::Ops& o);   // inst_weak_cvt.hip

bool pick_fp32_fp64_jets(int M, kern::Ops& o);   // inst_jets.hip

bool pick_fp32_fp64(int M, int walls, int weak, int cvt, kern::Ops& o)
{
  if ((walls & 3) == 3) return walls == 11 && !weak && !cvt && pick_fp32_fp64_jets(M, o);   // opposed jets
  if (weak && cvt) return pick_fp32_fp64_weak_cvt(M, walls, o);
  if (weak) return pick_fp32_fp64_weak(M, walls, o);
  if (cvt) return pick_fp32_fp64_cvt(M, walls, o);
  return kern::pick_m_any<float, double, float, false, false>(M, walls, o);
}
}  // namespace mclbm
