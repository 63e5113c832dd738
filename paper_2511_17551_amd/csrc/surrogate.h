// Temperature-guess surrogate: MLP 6 -> 64 -> 64 -> 64 -> 1 with tanh,
// BF16 MFMA operands and FP32 accumulation, FP32 master weights and Adam.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace dgx {

constexpr int kSurIn = 6;
constexpr int kSurH = 64;
// W1[64][6] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4[1]
constexpr int kSurParams = kSurH * kSurIn + kSurH + 2 * (kSurH * kSurH + kSurH) + kSurH + 1;
constexpr int kSurNorm = 14;  // feature mean[6], std[6], T mean, T std

struct Surrogate {
    bool ready = false;
    float *params = nullptr;  // device [kSurParams + kSurNorm] FP32 master copy
    float *adam_m = nullptr, *adam_v = nullptr, *grads = nullptr;
    int64_t step = 0;  // Adam steps taken
    std::string err;
};

int surrogate_set(Surrogate &S, const float *host_params);
int surrogate_get(Surrogate &S, float *host_params);
int surrogate_predict(Surrogate &S, int dim, const double *states, int64_t count, double *Tg, hipStream_t s);
int surrogate_train(Surrogate &S, int dim, const double *states, const double *T, int64_t count, int epochs,
                    int batch, float lr, uint64_t seed, float *loss_host, hipStream_t s);
int surrogate_grad(Surrogate &S, int dim, const double *states, const double *T, int64_t count, float *grad_host,
                   float *loss_host, hipStream_t s);
int surrogate_init(Surrogate &S, int dim, const double *states, const double *T, int64_t count, uint64_t seed,
                   hipStream_t s);
void surrogate_free(Surrogate &S);

}  // namespace dgx
