// Row-pass kernels (axis-2 r2c / c2r with the prologue and the general
// combine) instantiated for FP32 fields (the mixed-precision path).
#include "kernels_impl.hpp"
namespace ofdft {
OFDFT_INSTANTIATE_ROW(float)
}
