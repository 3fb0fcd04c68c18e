// nn_internal.hpp -- what the lattice context needs to know of a surrogate
// network (its channel count and tube sizes), for mclbm_nn_advance.
#pragma once

#include <vector>

#include "../../include/mclbm_nn.h"

namespace mclbm {
namespace nn {

// Channels, output form (species of the conservative output, 0 = direct) and
// [ntubes][3] tube sizes (nx, ny, nz) of a network.
void geometry(const mclbm_nn* net, int* channels, int* species, std::vector<int>* dims);

}  // namespace nn
}  // namespace mclbm
