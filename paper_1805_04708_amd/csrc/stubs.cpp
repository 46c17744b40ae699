// Entry points declared in jq.h whose subsystems are not part of this build
// yet: they validate nothing and report JQ_EUNSUPPORTED.
#include "internal.hpp"

extern "C" {
int jq_server_create(uint64_t, int, int, jq_encoding, jq_server** out) {
    if (out) *out = nullptr;
    jq::set_last_error("server is not built");
    return JQ_EUNSUPPORTED;
}
int jq_server_submit(jq_server*, const jq_circuit*, int, uint64_t*) { return JQ_EUNSUPPORTED; }
int jq_server_wait(jq_server*, int, jq_result*) { return JQ_EUNSUPPORTED; }
int jq_server_release(jq_server*, uint64_t) { return JQ_EUNSUPPORTED; }
int jq_server_stats_get(jq_server*, jq_server_stats*) { return JQ_EUNSUPPORTED; }
int jq_server_destroy(jq_server*) { return JQ_EUNSUPPORTED; }
}
