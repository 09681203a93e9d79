// Temporary: entry points not implemented yet.
#include "pcr_internal.h"
using namespace pcr;
extern "C" size_t pcr_reorder_scratch_bytes(uint64_t, int, uint32_t) { return 0; }
extern "C" int pcr_reorder(const pcr_point *, pcr_point *, uint32_t *, uint64_t, int, uint32_t, uint64_t, void *, size_t, void *) {
    return fail(PCR_EUNSUPPORTED, "reorder not built yet");
}
extern "C" int pcr_batch_create(pcr_batch **, const pcr_point *, uint64_t, uint32_t, const pcr_tune *, void *) {
    return fail(PCR_EUNSUPPORTED, "batch not built yet");
}
extern "C" int pcr_batch_launch(pcr_batch *, const pcr_view *, uint32_t, void *) { return fail(PCR_EUNSUPPORTED, "batch not built yet"); }
extern "C" int pcr_batch_destroy(pcr_batch *) { return PCR_OK; }
