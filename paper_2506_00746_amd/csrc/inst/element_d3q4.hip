// Element kernel and element-tangent kernel instantiations for D1 = 3 nodes
// and NQ = 4 Gauss points per direction (tangents on the FP64 matrix cores).
#include "../tangent_mfma.hpp"

namespace feod {
FEOD_INSTANTIATE_TANGENT_MFMA(4)
FEOD_INSTANTIATE(3, 4, fill_tangents_3_4)
}  // namespace feod
