// sam_sequence.cpp -- sequence and adjoint entry points (in progress).
#include "sam.h"

extern "C" {
sam_status sam_sequence_create(sam_ctx*, const sam_csc*, const sam_csc*, const sam_pattern_spec*, int32_t,
                               sam_precision, int32_t, sam_seq** seq, sam_stream_t) {
    if (seq) *seq = nullptr;
    return SAM_ERR_UNSUPPORTED;
}
sam_status sam_sequence_destroy(sam_seq*) { return SAM_OK; }
sam_status sam_sequence_info(const sam_seq*, int64_t*) { return SAM_ERR_UNSUPPORTED; }
sam_status sam_sequence_pattern(const sam_seq*, int32_t, const int32_t**, const int32_t**) { return SAM_ERR_UNSUPPORTED; }
sam_status sam_sequence_run(sam_seq*, const double* const*, void* const*, double*, sam_stream_t) {
    return SAM_ERR_UNSUPPORTED;
}
sam_status sam_backward(sam_plan*, const double*, const double*, const double*, double, double, sam_precision, double*,
                        double*, double*, double*, sam_stream_t) {
    return SAM_ERR_UNSUPPORTED;
}
}
