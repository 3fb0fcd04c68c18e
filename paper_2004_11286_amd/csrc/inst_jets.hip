// inst_jets.hip -- the opposed jets (nozzle inlets and free-slip walls on the x
// faces, outlets at the y ends) with FP64 storage and FP64 arithmetic, and with
// FP32 storage and FP64 arithmetic; strong coupling, constant properties.
#include "kernels.hpp"

namespace mclbm {
bool pick_fp64_jets(int M, kern::Ops& o) { return kern::pick_m_jets<double, double, double>(M, o); }
bool pick_fp32_fp64_jets(int M, kern::Ops& o) { return kern::pick_m_jets<float, double, float>(M, o); }
}  // namespace mclbm
