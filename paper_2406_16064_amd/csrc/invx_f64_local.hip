// Inverse-x pass kernels (double, demag off, uniform material): one
// translation unit per instantiation set, so that the library builds in parallel.
#include "hotpath.hpp"

namespace mmx {
template void inv_x_launch<double, false, false>(int, int, bool, const Launch<double>&, long long, int, size_t, hipStream_t);
}  // namespace mmx
