// Element kernel and element-tangent kernel instantiations for D1 = 3 nodes
// and NQ = 4 Gauss points per direction.
#include "../tangent_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE_TANGENT(3, 4)
FEOD_INSTANTIATE(3, 4, fill_tangents_3_4)
}  // namespace feod
