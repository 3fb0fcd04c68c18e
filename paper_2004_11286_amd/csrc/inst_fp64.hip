// inst_fp64.hip -- kernels with double storage and double arithmetic, double node record.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp64(int M, int walls, kern::Ops& o) { return kern::pick_m<double, double, double>(M, walls, o); }
}  // namespace mclbm
