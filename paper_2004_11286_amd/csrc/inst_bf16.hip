// inst_bf16.hip -- kernels with __bf16 storage and float arithmetic, float node record.
#include "kernels.hpp"

namespace mclbm {
bool pick_bf16(int M, int walls, kern::Ops& o) { return kern::pick_m<__bf16, float, float>(M, walls, o); }
}  // namespace mclbm
