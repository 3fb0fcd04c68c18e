// inst_fp32.hip -- kernels with float storage and float arithmetic.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp32(int M, int walls, kern::Ops& o) { return kern::pick_m<float, float>(M, walls, o); }
}  // namespace mclbm
