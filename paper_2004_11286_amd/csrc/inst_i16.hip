// inst_i16.hip -- kernels with 16-bit fixed-point storage (int16_t) and float
// arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
// strong and weak coupling with constant properties, periodic or walled x ends;
// open ends, free-slip walls and C_v(T) are compiled for FP64 arithmetic only
bool pick_i16(int M, int walls, int weak, int cvt, kern::Ops& o)
{
  if (cvt || walls > 1) return false;
  if (weak) return kern::pick_m<int16_t, float, float, true>(M, walls, o);
  return kern::pick_m<int16_t, float, float, false>(M, walls, o);
}
}  // namespace mclbm
