// qs_circuit.hip -- executing a gate list.
#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

Status run_gates(StateImpl* s, const std::vector<XGate>& gates, int flags) {
  (void)flags;
  for (const XGate& g : gates) {
    Status st = (g.control >= 0) ? launch_apply_cu(s, g.control, g.target, g.m)
                                 : launch_apply_1q(s, g.target, g.m);
    if (!st.good()) return st;
  }
  return Status::ok();
}

}  // namespace qs
