// Heuristic ADI shifts from Ritz values (Penzl's procedure).
#include "care.hpp"

namespace mpcare {

std::vector<Shift> penzl_shifts(Ctx* ctx, const SellOp& A64, int l0, int kp, int km) {
  (void)ctx;
  (void)A64;
  (void)l0;
  (void)kp;
  (void)km;
  fail(CARE_ERR_NOT_IMPLEMENTED, "automatic shift selection is not available yet; pass a shift set");
}

}  // namespace mpcare
