// Explicit instantiations: sddmm kernels on bf16 rows.
#include "kernels.h"

namespace spc3d {

template void launch_sddmm<bf16_t, 8>(SPC3D_SDDMM_LAUNCH_ARGS);
template void launch_sddmm<bf16_t, 1>(SPC3D_SDDMM_LAUNCH_ARGS);

}  // namespace spc3d
