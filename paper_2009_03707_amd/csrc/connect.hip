// placeholder, replaced below
#include "ctx.h"
namespace msc {
void connect_impl(ms_ctx* c, const uint32_t*, const Grid&, const uint32_t*, const int64_t*, ms_arcs* out) {
    memset(out, 0, sizeof(*out));
    fail(c, MS_ERR_INTERNAL, "connect not built yet");
}
}
