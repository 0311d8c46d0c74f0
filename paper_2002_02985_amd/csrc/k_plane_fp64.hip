// Plane kernels instantiated for FP64 fields.
#include "kernels_impl.hpp"
namespace ofdft {
#define PT double
OFDFT_INSTANTIATE_PLANES()
}
