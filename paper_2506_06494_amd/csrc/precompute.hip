// GPU precompute of the overshoot correction (placeholder until the band
// solver lands).
#include "jgs2_internal.h"

namespace jgs2 {
int precompute_device(jgs2_solver* s, int S, int n_cand, uint64_t seed) {
    (void)S; (void)n_cand; (void)seed;
    return s->fail(JGS2_E_INVALID, "GPU precompute not available in this build");
}
}  // namespace jgs2
