// Column-pass and per-knot kernels instantiated for FP32 fields (the mixed-precision path).
#include "kernels_impl.hpp"
namespace ofdft {
OFDFT_INSTANTIATE_COL(float)
}
