// qms_server.cpp -- the request loop (placeholder until the batched path lands).
#include "qms.h"
#include "qms_host.hpp"

using namespace qms;

extern "C" {
int qms_server_create(const qms_server_config *, qms_server **out) {
    if (out) *out = nullptr;
    return set_error(QMS_ERR_UNSUPPORTED, "server not built yet");
}
int qms_server_submit(qms_server *, void *, uint64_t, int, uint64_t *) {
    return set_error(QMS_ERR_UNSUPPORTED, "server not built yet");
}
int qms_server_poll(qms_server *, uint64_t, double *) {
    return set_error(QMS_ERR_UNSUPPORTED, "server not built yet");
}
int qms_server_get_stats(qms_server *, qms_server_stats *) {
    return set_error(QMS_ERR_UNSUPPORTED, "server not built yet");
}
int qms_server_destroy(qms_server *) { return QMS_OK; }
}
