// Near-field sums and gradients for rho = 1, and the entry points of the near
// field: both dispatch on NearArgs::real_exp to the form compiled here or to
// the real-exponent form (nearfield_real.hip).
#include "nearfield_kernels.h"

namespace nfs {

template hipError_t launch_nearfield_form<float, false>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_form<double, false>(const NearArgs<double>&, int, hipStream_t);

template <typename R>
hipError_t launch_nearfield(const NearArgs<R>& a, int nchunks, hipStream_t st) {
  return a.real_exp ? launch_nearfield_form<R, true>(a, nchunks, st) : launch_nearfield_form<R, false>(a, nchunks, st);
}
template hipError_t launch_nearfield<float>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield<double>(const NearArgs<double>&, int, hipStream_t);

template hipError_t launch_nearfield_grad_form<float, false>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_grad_form<double, false>(const NearArgs<double>&, int, hipStream_t);

template <typename R>
hipError_t launch_nearfield_grad(const NearArgs<R>& a, int nchunks, hipStream_t st) {
  return a.real_exp ? launch_nearfield_grad_form<R, true>(a, nchunks, st)
                    : launch_nearfield_grad_form<R, false>(a, nchunks, st);
}
template hipError_t launch_nearfield_grad<float>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_grad<double>(const NearArgs<double>&, int, hipStream_t);

}  // namespace nfs
