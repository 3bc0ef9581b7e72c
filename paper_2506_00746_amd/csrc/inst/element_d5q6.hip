// Element kernel and element-tangent kernel instantiations for D1 = 5 nodes
// and NQ = 6 Gauss points per direction.
#include "../tangent_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE_TANGENT(5, 6)
FEOD_INSTANTIATE(5, 6, fill_tangents_5_6)
}  // namespace feod
