// Float64 instantiation of the per-site passes.  Built with
// -ffp-contract=off: every product and sum rounds separately, in the order
// written in step_kernels.h.
#include "step_kernels.h"

namespace mlb {
template struct Launch<double>;
}
