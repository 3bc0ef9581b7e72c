// Element kernel and element-tangent kernel instantiations for D1 = 2 nodes
// and NQ = 2 Gauss points per direction.
#include "../tangent_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE_TANGENT(2, 2)
FEOD_INSTANTIATE(2, 2, fill_tangents_2_2)
}  // namespace feod
