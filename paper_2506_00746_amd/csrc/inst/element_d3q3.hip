// Element kernel instantiation for D1 = 3 nodes and NQ = 3 Gauss points per direction.
#include "../element_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE(3, 3)
}  // namespace feod
