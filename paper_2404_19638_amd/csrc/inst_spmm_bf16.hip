// Explicit instantiations: spmm kernels on bf16 rows.
#include "kernels.h"

namespace spc3d {

template void launch_spmm<bf16_t, 8, false>(SPC3D_SPMM_LAUNCH_ARGS);
template void launch_spmm<bf16_t, 1, false>(SPC3D_SPMM_LAUNCH_ARGS);

}  // namespace spc3d
