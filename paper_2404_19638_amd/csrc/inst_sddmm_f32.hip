// Explicit instantiations: sddmm kernels on f32 rows.
#include "kernels.h"

namespace spc3d {

template void launch_sddmm<float, 4>(SPC3D_SDDMM_LAUNCH_ARGS);
template void launch_sddmm<float, 1>(SPC3D_SDDMM_LAUNCH_ARGS);

}  // namespace spc3d
