// Inverse-x pass kernels (float, demag off, cell-based material): one
// translation unit per instantiation set, so that the library builds in parallel.
#include "hotpath.hpp"

namespace mmx {
template void inv_x_launch<float, false, true>(int, int, bool, const Launch<float>&, long long, int, size_t, hipStream_t);
}  // namespace mmx
