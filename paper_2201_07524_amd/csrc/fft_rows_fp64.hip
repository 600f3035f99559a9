// FFT row passes (R2C, C2R, the fused 1-D chain) on FP64 grids: the kernel
// instances for every grid size 2^2..2^12 (fft_kernels.h).  One translation
// unit per kernel family and precision, so the instances compile in parallel.
#include "fft_kernels.h"

namespace nfs {
template hipError_t launch_rows<double>(const RowArgs<double>&, hipStream_t);
}  // namespace nfs
