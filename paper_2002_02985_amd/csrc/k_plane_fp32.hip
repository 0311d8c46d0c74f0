// Plane kernels instantiated for FP32 fields.
#include "kernels_impl.hpp"
namespace ofdft {
#define PT float
OFDFT_INSTANTIATE_PLANES()
}
