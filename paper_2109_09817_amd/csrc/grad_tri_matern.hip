// Matern-5/2 instantiations of the upper-triangle hyperparameter-form sweep.
#include "grad_tri_impl.h"

namespace gpk {

int grad_tri_ksc(int t) {
  const int need = (6 * t + 31) / 32;
  static const int kAvail[] = {1, 2, 3, 4, 6, 8, 12};
  for (int k : kAvail)
    if (k >= need) return k;
  return -1;
}

bool launch_grad_tri_matern(int ks, int nj, int ksc, unsigned units, const GradTriArgs& a, hipStream_t st) {
  return tri_dispatch<GP_MATERN52>(ks, nj, ksc, units, a, st);
}

}  // namespace gpk
