// Element kernel instantiation for D1 = 4 nodes and NQ = 5 Gauss points per direction.
#include "../element_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE(4, 5)
}  // namespace feod
