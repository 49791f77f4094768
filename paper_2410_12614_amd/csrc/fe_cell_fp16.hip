// Cell-kernel and fused-assembly instantiations for one precision
// (see fe_cell_kernel.h and fe_fused.h).
#include "fe_cell_kernel.h"
#include "fe_cellwise.h"
#include "fe_fused.h"
#include "fe_smallcell.h"

namespace fe {
fe_status launch_cell_fp16(const CellLaunch &a) { return launch_cell_impl<PolF16>(a); }
fe_status launch_fused_fp16(const FusedLaunch &a) { return launch_fused_impl<PolF16>(a); }
fe_status launch_cellwise_fp16(const CellwiseLaunch &c) { return launch_cellwise(c); }
fe_status launch_small_fp16(const CellLaunch &a) { return launch_small(a); }
}  // namespace fe
