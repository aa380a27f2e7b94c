// Float32 instantiation of the per-site passes (contraction allowed).
#include "step_kernels.h"

namespace mlb {
template struct Launch<float>;
}
