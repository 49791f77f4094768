// Cell-kernel and fused-assembly instantiations for one precision
// (see fe_cell_kernel.h and fe_fused.h).
#include "fe_cell_kernel.h"
#include "fe_fused.h"

namespace fe {
fe_status launch_cell_bf16(const CellLaunch &a) { return launch_cell_impl<PolBF16>(a); }
fe_status launch_fused_bf16(const FusedLaunch &a) { return launch_fused_impl<PolBF16>(a); }
}  // namespace fe
