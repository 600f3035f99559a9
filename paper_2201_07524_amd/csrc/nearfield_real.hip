// Near-field sums and gradients for a real cost exponent rho: the kernel
// exp(-r^rho/eps) with r^rho = (r^2)^(rho/2) (launch_nearfield and
// launch_nearfield_grad dispatch here when NearArgs::real_exp is set).
#include "nearfield_kernels.h"

namespace nfs {

template hipError_t launch_nearfield_form<float, kNearReal>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_form<double, kNearReal>(const NearArgs<double>&, int, hipStream_t);
template hipError_t launch_nearfield_grad_form<float, kNearReal>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_grad_form<double, kNearReal>(const NearArgs<double>&, int, hipStream_t);

}  // namespace nfs
