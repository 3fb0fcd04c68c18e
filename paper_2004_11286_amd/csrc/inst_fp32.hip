// inst_fp32.hip -- kernels with float storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp32(int M, int walls, kern::Ops& o) { return kern::pick_m<float, float, float>(M, walls, o); }
}  // namespace mclbm
