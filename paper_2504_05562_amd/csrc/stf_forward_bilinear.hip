// Forward kernels of the bilinear filter (one-tap, quad, record and
// whole-tile exchange; 1-4 textures; with and without the latent decoder
// and exact filtering), instantiated here so they compile apart from the
// rest of the library.
#include "stf_kernels.h"

namespace stf {

template void launch_forward<0, kModeStf>(const Args&, hipStream_t);
template void launch_forward<0, kModeQuad>(const Args&, hipStream_t);
template void launch_forward<0, kModeRecords>(const Args&, hipStream_t);
template void launch_forward<0, kModeBins>(const Args&, hipStream_t);

}  // namespace stf
