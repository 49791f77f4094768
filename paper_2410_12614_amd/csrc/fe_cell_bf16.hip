// Cell-kernel instantiations for one precision (see fe_cell_kernel.h).
#include "fe_cell_kernel.h"

namespace fe {
fe_status launch_cell_bf16(const CellLaunch &a) { return launch_cell_impl<PolBF16>(a); }
}  // namespace fe
