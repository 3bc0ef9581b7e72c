// Element kernel and element-tangent kernel instantiations for D1 = 3 nodes
// and NQ = 3 Gauss points per direction (tangents on the FP64 matrix cores).
#include "../tangent_mfma.hpp"

namespace feod {
FEOD_INSTANTIATE_TANGENT_MFMA(3)
FEOD_INSTANTIATE(3, 3, fill_tangents_3_3)
}  // namespace feod
