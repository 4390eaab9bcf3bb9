// mid_f32.hip -- the last-axis pass with the spectral product in single precision,
// compiled apart from the rest of the pipeline so the builds run in parallel.
#include "passes.h"

namespace mmx {
MMX_MID_INST(, float)
}  // namespace mmx
