// inst_fp16.hip -- kernels with _Float16 storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp16(int M, int walls, kern::Ops& o) { return kern::pick_m<_Float16, float, float>(M, walls, o); }
}  // namespace mclbm
