// Element kernel and element-tangent kernel instantiations for D1 = 3 nodes
// and NQ = 3 Gauss points per direction.
#include "../tangent_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE_TANGENT(3, 3)
FEOD_INSTANTIATE(3, 3, fill_tangents_3_3)
}  // namespace feod
