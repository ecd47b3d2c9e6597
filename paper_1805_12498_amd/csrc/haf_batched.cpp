// Batched hafnians (one persistent launch over many matrices).
#include "haf_runtime.hpp"

using namespace hafgpu;

extern "C" int haf_batched_c128(const haf_cplx* dA_packed, const int64_t* h_offsets, const int32_t* h_n,
                                const uint8_t* h_kind, int count, haf_cplx* d_out, void* stream) {
    (void)dA_packed; (void)h_offsets; (void)h_n; (void)h_kind; (void)count; (void)d_out; (void)stream;
    clear_error();
    return set_error(HAF_E_STATE, "batched path not available in this build");
}
