// Row-pass combine kernels with fixed term sets, FP32 fields (the mixed-precision path).
#include "kernels_impl.hpp"
namespace ofdft {
OFDFT_INSTANTIATE_ROW_FIXED(float)
}
