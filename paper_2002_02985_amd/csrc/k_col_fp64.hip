// Column-pass and per-knot kernels instantiated for FP64 fields (the plain FP64 path).
#include "kernels_impl.hpp"
namespace ofdft {
OFDFT_INSTANTIATE_COL(double)
}
