// Surrogate MLP kernels (placeholder until the MFMA kernels land).
#include "rd_mlp.hpp"

namespace rd {

struct Surrogate {
    int dummy;
};

int32_t surrogate_new(Surrogate **out, const SurrogateDesc &, uint32_t)
{
    *out = nullptr;
    return -4;
}
void surrogate_destroy(Surrogate *s) { delete s; }
bool surrogate_ready(const Surrogate *) { return false; }
int surrogate_max_batch(const Surrogate *) { return 0; }
int surrogate_layers(const Surrogate *) { return 0; }
hipError_t surrogate_downsample(Surrogate *, int, const void *, float *, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t surrogate_scaling(Surrogate *, const float *, const float *, double, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t surrogate_train(Surrogate *, int, const double *, const float *, double, double *,
                           hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t surrogate_predict(Surrogate *, int, const double *, float *, int, hipStream_t)
{
    return hipErrorNotSupported;
}
int32_t surrogate_enqueue_loglik(Surrogate *, int, const double *, double *, hipStream_t)
{
    return -4;
}
hipError_t surrogate_copy_params(Surrogate *, int, float *, float *, int, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace rd
