// Element kernel instantiation for D1 = 2 nodes and NQ = 2 Gauss points per direction.
#include "../element_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE(2, 2)
}  // namespace feod
