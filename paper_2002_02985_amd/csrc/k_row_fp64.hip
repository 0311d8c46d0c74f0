// Row-pass kernels (axis-2 r2c / c2r with the prologue and the general
// combine) instantiated for FP64 fields (the plain FP64 path).
#include "kernels_impl.hpp"
namespace ofdft {
OFDFT_INSTANTIATE_ROW(double)
}
