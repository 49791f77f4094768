// Action-kernel instantiations for double precision (see fe_action.h).
#include "fe_action.h"

namespace fe {
fe_status launch_action_fp64(const ActionLaunch &a) { return launch_action_impl<PolF64>(a); }
}  // namespace fe
