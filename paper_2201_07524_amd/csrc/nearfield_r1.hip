// Near-field sums and gradients for rho = 1, and the entry points of the near
// field: both dispatch on NearArgs::cost and NearArgs::real_exp to the form
// compiled here, the real-exponent form (nearfield_real.hip) or the primal
// cost's kernel (nearfield_cost.hip, sums only).
#include "nearfield_kernels.h"

namespace nfs {

template hipError_t launch_nearfield_form<float, kNearR1>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_form<double, kNearR1>(const NearArgs<double>&, int, hipStream_t);

template <typename R>
hipError_t launch_nearfield(const NearArgs<R>& a, int nchunks, hipStream_t st) {
  if (a.cost) return launch_nearfield_form<R, kNearCost>(a, nchunks, st);
  return a.real_exp ? launch_nearfield_form<R, kNearReal>(a, nchunks, st)
                    : launch_nearfield_form<R, kNearR1>(a, nchunks, st);
}
template hipError_t launch_nearfield<float>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield<double>(const NearArgs<double>&, int, hipStream_t);

template hipError_t launch_nearfield_grad_form<float, kNearR1>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_grad_form<double, kNearR1>(const NearArgs<double>&, int, hipStream_t);

template <typename R>
hipError_t launch_nearfield_grad(const NearArgs<R>& a, int nchunks, hipStream_t st) {
  if (a.cost) return hipErrorInvalidValue;  // no gradient of the primal cost's kernel
  return a.real_exp ? launch_nearfield_grad_form<R, kNearReal>(a, nchunks, st)
                    : launch_nearfield_grad_form<R, kNearR1>(a, nchunks, st);
}
template hipError_t launch_nearfield_grad<float>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_grad<double>(const NearArgs<double>&, int, hipStream_t);

}  // namespace nfs
