// Row-pass combine kernels with fixed term sets, FP64 fields (the plain FP64 path).
#include "kernels_impl.hpp"
namespace ofdft {
OFDFT_INSTANTIATE_ROW_FIXED(double)
}
