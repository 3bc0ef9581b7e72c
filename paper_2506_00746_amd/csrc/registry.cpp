// Table of compiled (D1, NQ) element-kernel instantiations.
#include "kernel_api.hpp"

namespace feod {

#define FEOD_PAIRS(X) X(2, 2) X(3, 3) X(3, 4) X(4, 5) X(5, 6) X(8, 9)

#define FEOD_DECLARE(D1, NQ) ElemLaunchers make_launchers_##D1##_##NQ();
FEOD_PAIRS(FEOD_DECLARE)

const ElemLaunchers* find_launchers(int D1, int NQ) {
#define FEOD_ENTRY(D1, NQ) make_launchers_##D1##_##NQ(),
  static const ElemLaunchers table[] = {FEOD_PAIRS(FEOD_ENTRY)};
  for (const auto& t : table)
    if (t.D1 == D1 && t.NQ == NQ) return &t;
  return nullptr;
}

}  // namespace feod
