// Near-field sums of the primal cost's kernel |z|^rho exp(-|z|^rho/eps) (the
// cost-weighted kernel of <pi, C>, eq. (15)) for r = 1 and real exponents:
// launch_nearfield dispatches here when NearArgs::cost is set.
#include "nearfield_kernels.h"

namespace nfs {

template hipError_t launch_nearfield_form<float, kNearCost>(const NearArgs<float>&, int, hipStream_t);
template hipError_t launch_nearfield_form<double, kNearCost>(const NearArgs<double>&, int, hipStream_t);

}  // namespace nfs
