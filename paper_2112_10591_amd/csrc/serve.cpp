// serve.cpp -- serving runtime (placeholder until the batch former lands).
#include "ctx.h"

namespace ebof {
struct ServeState {};
void serve_shutdown(ebof_ctx*) {}
}  // namespace ebof

using namespace ebof;

extern "C" {
int ebof_stream_open(ebof_ctx*, const ebof_params*, int32_t*) { set_error("serving not built"); return EBOF_E_STATE; }
int ebof_stream_close(ebof_ctx*, int32_t) { set_error("serving not built"); return EBOF_E_STATE; }
int ebof_submit(ebof_ctx*, int32_t, const uint16_t*, const uint16_t*, const int64_t*, int64_t, int64_t, int, float*,
                uint8_t*, uint64_t*) { set_error("serving not built"); return EBOF_E_STATE; }
int ebof_poll(ebof_ctx*, uint64_t, int32_t*) { set_error("serving not built"); return EBOF_E_STATE; }
int ebof_drain(ebof_ctx*) { return EBOF_OK; }
}
