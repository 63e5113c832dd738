// Surrogate MLP kernels (filled in below).
#include "surrogate.h"

namespace dgx {

int surrogate_set(Surrogate &S, const float *host_params) {
    if (!S.params && hipMalloc(&S.params, (kSurParams + kSurNorm) * sizeof(float)) != hipSuccess) return -3;
    if (hipMemcpy(S.params, host_params, (kSurParams + kSurNorm) * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return -3;
    S.ready = true;
    return 0;
}
int surrogate_get(Surrogate &S, float *host_params) {
    return hipMemcpy(host_params, S.params, (kSurParams + kSurNorm) * sizeof(float), hipMemcpyDeviceToHost) ==
                   hipSuccess ? 0 : -3;
}
int surrogate_predict(Surrogate &, int, const double *, int64_t, double *, hipStream_t) { return -3; }
int surrogate_train(Surrogate &S, int, const double *, const double *, int64_t, int, int, float, uint64_t, float *,
                    hipStream_t) {
    S.err = "not built";
    return -3;
}
void surrogate_free(Surrogate &S) {
    if (S.params) (void)hipFree(S.params);
    if (S.adam_m) (void)hipFree(S.adam_m);
    if (S.adam_v) (void)hipFree(S.adam_v);
    if (S.grads) (void)hipFree(S.grads);
    S = Surrogate();
}

}  // namespace dgx
