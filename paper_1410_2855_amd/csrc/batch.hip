// batch.hip -- placeholder until the persistent batched kernel lands.
#include "host.hpp"

using namespace lsr;

extern "C" {
int lsr_batch_create(lsr_batch* out, const lsr_plan*, int) {
    if (out) *out = nullptr;
    return set_err(LSR_EUNSUPPORTED, "batching not built yet");
}
int lsr_batch_roundtrips(lsr_batch, void* const*, void* const*, int) { return set_err(LSR_EUNSUPPORTED, "batching not built yet"); }
int lsr_batch_diag(lsr_batch, int, const void*, const void*, lsr_diag_out*) { return set_err(LSR_EUNSUPPORTED, "batching not built yet"); }
int lsr_batch_set_graph_trips(lsr_batch, int) { return set_err(LSR_EUNSUPPORTED, "batching not built yet"); }
void lsr_batch_destroy(lsr_batch) {}
int lsr_autotune(lsr_plan, lsr_batch, const char*) { return set_err(LSR_EUNSUPPORTED, "autotune not built yet"); }
int lsr_pack_tasks(const int*, int, int, int*, int) { return set_err(LSR_EUNSUPPORTED, "batching not built yet"); }
}
