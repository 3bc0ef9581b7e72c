// Element kernel instantiation for D1 = 5 nodes and NQ = 6 Gauss points per direction.
#include "../element_kernel.hpp"

namespace feod {
FEOD_INSTANTIATE(5, 6)
}  // namespace feod
