// Continuous-batching request server.
#include "haf_runtime.hpp"

using namespace hafgpu;

extern "C" {
void haf_server_default_config(haf_server_config* cfg) {
    if (!cfg) return;
    cfg->device = 0;
    cfg->arena_bytes = (int64_t)1 << 30;
    cfg->max_active = 256;
    cfg->max_queue = 1 << 20;
    cfg->tick_units = 4096;
    cfg->continuous = 1;
}
haf_server* haf_server_create(const haf_server_config* cfg) { (void)cfg; set_error(HAF_E_STATE, "server not available in this build"); return nullptr; }
int haf_server_submit(haf_server* s, const haf_cplx* A, int n, int lda, int kind, uint64_t* ticket) { (void)s; (void)A; (void)n; (void)lda; (void)kind; (void)ticket; return set_error(HAF_E_STATE, "server not available"); }
int haf_server_poll(haf_server* s, haf_result* out, int max, int* n_out) { (void)s; (void)out; (void)max; (void)n_out; return set_error(HAF_E_STATE, "server not available"); }
int haf_server_drain(haf_server* s) { (void)s; return set_error(HAF_E_STATE, "server not available"); }
void haf_server_destroy(haf_server* s) { (void)s; }
}
