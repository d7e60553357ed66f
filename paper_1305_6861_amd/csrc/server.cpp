// Batched and served execution (persistent work-queue kernel, request loop).
#include "ps_runtime.h"

namespace ps {

void destroy_runtime(Ctx*) {}

}  // namespace ps
