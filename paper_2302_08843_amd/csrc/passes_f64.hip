// passes_f64.hip -- x and y passes and the plain local pass in double precision,
// compiled apart from the rest of the pipeline so the builds run in parallel.
#include "passes.h"

namespace mmx {
MMX_PASS_INST(, double)
}  // namespace mmx
