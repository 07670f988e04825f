// Explicit instantiations: fused kernels on f32 rows.
#include "kernels.h"

namespace spc3d {

template void launch_spmm<float, 4, true>(SPC3D_SPMM_LAUNCH_ARGS);
template void launch_spmm<float, 1, true>(SPC3D_SPMM_LAUNCH_ARGS);

}  // namespace spc3d
