// inst_fp16.hip -- kernels with _Float16 storage and float arithmetic.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp16(int M, int walls, kern::Ops& o) { return kern::pick_m<_Float16, float>(M, walls, o); }
}  // namespace mclbm
