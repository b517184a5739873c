// Required number of moduli (Theorem 1, eq. thm:err-2).  Placeholder until
// the lower-bound product kernel exists: reports an argument error.
#include "../../include/ozaki2.h"

extern "C" int ozaki2_required_moduli(int prec, int m, int n, int k, const void* A, int lda,
                                      const void* B, int ldb, double eps, int* N_out) {
  (void)prec; (void)m; (void)n; (void)k; (void)A; (void)lda; (void)B; (void)ldb; (void)eps;
  if (N_out) *N_out = 0;
  return OZAKI2_ERR_INVALID_ARG;
}
