// Surrogate MLP (first stage of delayed acceptance): internal interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rd {

struct SurrogateDesc {
    int width;        // hidden width
    int depth;        // hidden layers
    int out_side;     // side of the downsampled field
    int n;            // side of the full grid
    int precision;    // precision of full-grid fields passed to downsample
    double lo[4], hi[4];
    const double *y;  // full-grid data (device, float64)
    int max_batch;
};

struct SurScale {
    double lo[4], hi[4];
};

struct Surrogate;

int32_t surrogate_new(Surrogate **out, const SurrogateDesc &d, uint32_t seed);
void surrogate_destroy(Surrogate *s);
bool surrogate_ready(const Surrogate *s);
int surrogate_max_batch(const Surrogate *s);
int surrogate_layers(const Surrogate *s);
hipError_t surrogate_downsample(Surrogate *s, int n, const void *u, float *out, hipStream_t st);
void surrogate_input_box(Surrogate *s, const double lo[4], const double hi[4]);
hipError_t surrogate_scaling(Surrogate *s, const float *mean, const float *sd, double sigma1,
                             hipStream_t st);
hipError_t surrogate_train(Surrogate *s, int batch, const double *phi, const float *target,
                           double lr, double *loss, hipStream_t st);
hipError_t surrogate_predict(Surrogate *s, int n, const double *phi, float *out, int raw,
                             hipStream_t st);
int32_t surrogate_enqueue_loglik(Surrogate *s, int n, const double *phi, double *ll, hipStream_t st);
hipError_t surrogate_copy_params(Surrogate *s, int layer, float *w, float *b, int dir,
                                 hipStream_t st);

}  // namespace rd
