// Element kernel and element-tangent kernel instantiations for D1 = 4 nodes
// and NQ = 5 Gauss points per direction.
#include "../tangent_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE_TANGENT(4, 5)
FEOD_INSTANTIATE(4, 5, fill_tangents_4_5)
}  // namespace feod
