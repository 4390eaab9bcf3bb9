// local_ext_f64.hip -- the extended stencil variants of the x inverse / local
// pass (DMI, per-cell exchange, DMI and uniaxial constants) in double precision, compiled
// apart from the rest of the pipeline so the builds run in parallel.
#include "passes.h"

namespace mmx {
template hipError_t launch_local_ext<double>(const Plan&, int, const double*, double*, double*, const LocalParams&,
                                          double*, bool, int);
}  // namespace mmx
