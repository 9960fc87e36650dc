// Batched path (placeholder until the persistent queue lands).
#include "lacosmic_internal.h"
namespace lac {
void DevCtx::release_extras() {}
}
