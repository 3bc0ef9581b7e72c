// Element kernel instantiation for D1 = 8 nodes and NQ = 9 Gauss points per direction.
#include "../element_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE(8, 9)
}  // namespace feod
