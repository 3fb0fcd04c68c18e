// inst_fp32_fp64.hip -- kernels with float storage and double arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp32_fp64(int M, int walls, kern::Ops& o) { return kern::pick_m<float, double, float>(M, walls, o); }
}  // namespace mclbm
