// FFT strided axis passes on FP64 grids: the kernel
// instances for every grid size 2^2..2^12 (fft_kernels.h).  One translation
// unit per kernel family and precision, so the instances compile in parallel.
#include "fft_kernels.h"

namespace nfs {
template hipError_t launch_axis<double>(const AxisArgs<double>&, hipStream_t);
}  // namespace nfs
