// passes_f32.hip -- x and y passes and the plain local pass in single precision,
// compiled apart from the rest of the pipeline so the builds run in parallel.
#include "passes.h"

namespace mmx {
MMX_PASS_INST(, float)
}  // namespace mmx
