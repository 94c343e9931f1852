// server.hip -- serving loop (in progress: entry points report INVALID).
#include "fmm_internal.h"

extern "C" {
fmm_status fmm_server_create(const fmm_server_options *, fmm_server_t *out)
{
    if (out) *out = nullptr;
    fmm::set_error("serving not built yet");
    return FMM_E_INVALID;
}
fmm_status fmm_submit(fmm_server_t, const fmm_request *, uint64_t *) { return FMM_E_INVALID; }
fmm_status fmm_poll(fmm_server_t, uint64_t, double *, fmm_result *) { return FMM_E_INVALID; }
fmm_status fmm_server_drain(fmm_server_t) { return FMM_E_INVALID; }
fmm_status fmm_server_destroy(fmm_server_t) { return FMM_E_INVALID; }
}
