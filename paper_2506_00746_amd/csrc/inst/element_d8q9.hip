// Element kernel instantiation for D1 = 8 nodes and NQ = 9 Gauss points per
// direction (no element-tangent kernel: its LDS stage exceeds the CU's LDS).
#include "../element_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE(8, 9, no_tangents)
}  // namespace feod
