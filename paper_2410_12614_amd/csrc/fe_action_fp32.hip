// Action-kernel instantiations for single precision (see fe_action.h).
#include "fe_action.h"

namespace fe {
fe_status launch_action_fp32(const ActionLaunch &a) { return launch_action_impl<PolF32>(a); }
}  // namespace fe
