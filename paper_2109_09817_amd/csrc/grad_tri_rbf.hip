// RBF instantiations of the upper-triangle hyperparameter-form sweep.
#include "grad_tri_impl.h"

namespace gpk {

bool launch_grad_tri_rbf(int ks, int nj, int ksc, unsigned units, const GradTriArgs& a, hipStream_t st) {
  return tri_dispatch<GP_RBF>(ks, nj, ksc, units, a, st);
}

}  // namespace gpk
