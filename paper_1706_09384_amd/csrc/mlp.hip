// Rank-model entry points (filled in by the MLP implementation).
#include "internal.hpp"

extern "C" hm_status hm_rank_samples(const hm_matrix *, float *, int32_t *) { return HM_ERR_STATE; }
extern "C" hm_status hm_rank_model_train(const float *, const int32_t *, int64_t, float *, int32_t,
                                         int32_t, float, uint64_t, float *, void *) {
    return HM_ERR_STATE;
}
extern "C" hm_status hm_rank_model_predict(const float *, const float *, float *, int64_t, void *) {
    return HM_ERR_STATE;
}
extern "C" hm_status hm_rank_model_grad(const float *, const float *, const float *, int64_t, float *,
                                        float *, void *) {
    return HM_ERR_STATE;
}
