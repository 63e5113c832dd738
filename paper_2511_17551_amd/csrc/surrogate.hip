// Temperature-guess surrogate: a 6 -> 64 -> 64 -> 64 -> 1 tanh MLP on the
// BF16 matrix cores of gfx950 (v_mfma_f32_16x16x16_bf16, FP32 accumulation),
// FP32 master weights, Adam.  It supplies the initial guess of the per-node
// T(e) Newton iteration (Appendix, Thermodynamics; the Introduction's
// requirement that the iterative thermochemistry be cheap).
//
// Wave-level tiling: a wave processes 16 samples.  With the MFMA operand
// layout (lane l, group g = l/16, row r = l%16)
//   A[m = r][k = 4g + j],  B[k = 4g + j][n = r],  D[m = 4g + j][n = r]  (j = 0..3)
// weights are the A operand (neurons x inputs) and activations the B operand
// (inputs x samples); a layer's FP32 result D, after bias + tanh and rounding
// to BF16, is exactly the B operand of the next layer (K block = output block).
// Weight gradients dW = dz . h^T contract over samples and take their
// operands through a per-wave LDS transpose.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "surrogate.h"

namespace dgx {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int H = kSurH;
// parameter offsets
constexpr int oW1 = 0, ob1 = oW1 + H * kSurIn, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H,
              ob3 = oW3 + H * H, oW4 = ob3 + H, ob4 = oW4 + H, oNorm = ob4 + 1;
static_assert(oNorm == kSurParams, "parameter layout");

// FP32 -> BF16, round to nearest even: the conversion instruction of gfx950
// (v_cvt_pk_bf16_f32, which also packs pairs)
__device__ __forceinline__ unsigned short to_bf16(float f) {
    return __builtin_bit_cast(unsigned short, (__bf16)f);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef unsigned u32x2v __attribute__((ext_vector_type(2)));

// Four floats to BF16 (round to nearest even) in two paired conversions, one
// per dword, so that no byte shuffles are needed to assemble the fragment.
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    const f32x2v lo = {a, b}, hi = {c, d};
    const u32x2v w = {__builtin_bit_cast(unsigned, __builtin_convertvector(lo, bf16x2v)),
                      __builtin_bit_cast(unsigned, __builtin_convertvector(hi, bf16x2v))};
    return __builtin_bit_cast(bf16x4, w);
}

// tanh(x) = 1 - 2 / (exp(2x) + 1) with the hardware exp and reciprocal
// estimates (v_exp_f32, v_rcp_f32: FP32, about one ulp each; the activations
// are rounded to BF16 right after, or feed the FP32 output layer).
__device__ __forceinline__ float tanh_fast(float x) {
    const float t = __expf(2.0f * x);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(t + 1.0f);
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Standardised features of sample i (packed states [nvar][count]):
// log10 max(rho_s, 1e-30) for the 5 species and the specific internal energy.
template <int DIM>
__device__ __forceinline__ void features(const double *st, int64_t count, int64_t i, const float *nrm,
                                         float *x) {
    double rs[5], rho = 0.0;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        rs[s] = st[s * count + i];
        rho += rs[s];
    }
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double m = st[(5 + c) * count + i];
        m2 += m * m;
    }
    // the specific energy in FP64 (kinetic energy can dominate E); the
    // logarithms and the standardisation in FP32, which the features are
    // rounded to (and then to BF16 for the matrix unit)
    const double e = (st[(5 + DIM) * count + i] - 0.5 * m2 / rho) / rho;
#pragma unroll
    for (int s = 0; s < 5; ++s) x[s] = (log10f(fmaxf((float)rs[s], 1e-30f)) - nrm[s]) / nrm[6 + s];
    x[5] = (float)((e - (double)nrm[5]) / (double)nrm[11]);
}

// A fragment of a weight matrix W[rows][ld] (FP32 master) for output block
// mt and input block kc, rounded to BF16; columns >= ncol read as 0.
__device__ __forceinline__ bf16x4 wfrag(const float *W, int ld, int ncol, int mt, int kc, int r, int g) {
    float v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = 16 * kc + 4 * g + j;
        v[j] = col < ncol ? W[(16 * mt + r) * ld + col] : 0.0f;
    }
    return pack4(v[0], v[1], v[2], v[3]);
}
// A fragment of W^T (input block mt as rows, output block kc as K).
__device__ __forceinline__ bf16x4 wtfrag(const float *W, int ld, int mt, int kc, int r, int g) {
    float v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = W[(16 * kc + 4 * g + j) * ld + 16 * mt + r];
    return pack4(v[0], v[1], v[2], v[3]);
}

struct Fwd {
    float h1[4][4], h2[4][4], h3[4][4];  // FP32 activations, D layout
    bf16x4 hb1[4], hb2[4];               // BF16 B-operands of layers 2 and 3
    bf16x4 xb;                           // BF16 features (B operand of layer 1)
    float y;                             // output before b4 (summed over groups)
};

__device__ __forceinline__ void forward(const float *P, const float *x, int r, int g, Fwd &F) {
    {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            v[j] = k < 6 ? x[k] : 0.0f;
        }
        F.xb = pack4(v[0], v[1], v[2], v[3]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(wfrag(P + oW1, kSurIn, kSurIn, mt, 0, r, g), F.xb, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) F.h1[mt][j] = tanh_fast(acc[j] + P[ob1 + 16 * mt + 4 * g + j]);
        F.hb1[mt] = pack4(F.h1[mt][0], F.h1[mt][1], F.h1[mt][2], F.h1[mt][3]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) acc = mfma(wfrag(P + oW2, H, H, mt, kc, r, g), F.hb1[kc], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) F.h2[mt][j] = tanh_fast(acc[j] + P[ob2 + 16 * mt + 4 * g + j]);
        F.hb2[mt] = pack4(F.h2[mt][0], F.h2[mt][1], F.h2[mt][2], F.h2[mt][3]);
    }
    float yp = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) acc = mfma(wfrag(P + oW3, H, H, mt, kc, r, g), F.hb2[kc], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            F.h3[mt][j] = tanh_fast(acc[j] + P[ob3 + 16 * mt + 4 * g + j]);
            yp = fmaf(P[oW4 + 16 * mt + 4 * g + j], F.h3[mt][j], yp);
        }
    }
    yp += __shfl_xor(yp, 16);
    yp += __shfl_xor(yp, 32);
    F.y = yp;
}

// ------------------------------------------------------------ inference
// Weight fragments stay in registers for the whole kernel; biases and W4 sit
// in LDS; the features of 64 samples are computed one sample per lane and
// shared through LDS by the four 16-sample tiles.
template <int DIM>
__global__ void __launch_bounds__(256) k_mlp_predict(const float *__restrict__ P, const double *__restrict__ st,
                                                     int64_t count, double *__restrict__ Tg) {
    __shared__ float sx[4][64][8];         // per wave: features of 64 samples
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const float *nrm = P + oNorm;
    bf16x4 W1f[4], W2f[4][4], W3f[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        W1f[mt] = wfrag(P + oW1, kSurIn, kSurIn, mt, 0, r, g);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            W2f[mt][kc] = wfrag(P + oW2, H, H, mt, kc, r, g);
            W3f[mt][kc] = wfrag(P + oW3, H, H, mt, kc, r, g);
        }
    }
    // this lane's biases (rows 16 mt + 4 g + j) start the accumulators, and
    // its output weights W4
    f32x4 bias1[4], bias2[4], bias3[4], w4[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 16 * mt + 4 * g + j;
            bias1[mt][j] = P[ob1 + row];
            bias2[mt][j] = P[ob2 + row];
            bias3[mt][j] = P[ob3 + row];
            w4[mt][j] = P[oW4 + row];
        }
    const float b4 = P[ob4];
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t s0 = wave * 64; s0 < count; s0 += nwaves * 64) {
        {
            float x[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (s0 + lane < count) features<DIM>(st, count, s0 + lane, nrm, x);
#pragma unroll
            for (int k = 0; k < 6; ++k) sx[w][lane][k] = x[k];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // two independent 16-sample tiles per pass: the matrix unit works on
        // one while the vector ALU evaluates the other's tanh
#pragma unroll 1
        for (int tt = 0; tt < 4; tt += 2) {
            bf16x4 xb[2];
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) {
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 4 * g + j;
                    v[j] = k < 6 ? sx[w][16 * (tt + t2) + r][k] : 0.0f;
                }
                xb[t2] = pack4(v[0], v[1], v[2], v[3]);
            }
            bf16x4 hb[2][4], hc[2][4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
                for (int t2 = 0; t2 < 2; ++t2) {
                    const f32x4 acc = mfma(W1f[mt], xb[t2], bias1[mt]);
                    float h[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) h[j] = tanh_fast(acc[j]);
                    hb[t2][mt] = pack4(h[0], h[1], h[2], h[3]);
                }
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
                for (int t2 = 0; t2 < 2; ++t2) {
                    f32x4 acc = bias2[mt];
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) acc = mfma(W2f[mt][kc], hb[t2][kc], acc);
                    float h[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) h[j] = tanh_fast(acc[j]);
                    hc[t2][mt] = pack4(h[0], h[1], h[2], h[3]);
                }
            }
            float yp[2] = {0.0f, 0.0f};
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
                for (int t2 = 0; t2 < 2; ++t2) {
                    f32x4 acc = bias3[mt];
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) acc = mfma(W3f[mt][kc], hc[t2][kc], acc);
#pragma unroll
                    for (int j = 0; j < 4; ++j) yp[t2] = fmaf(w4[mt][j], tanh_fast(acc[j]), yp[t2]);
                }
            }
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) {
                float y = yp[t2];
                y += __shfl_xor(y, 16);
                y += __shfl_xor(y, 32);
                const int64_t n = s0 + 16 * (tt + t2) + r;
                if (g == 0 && n < count) Tg[n] = (double)(y + b4) * (double)nrm[13] + (double)nrm[12];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ------------------------------------------------------------ training
// Per-block partial gradients of the mean squared error over the samples
// idx[start + b*spb .. start + (b+1)*spb) (b = block), spb = 4 waves x tpw tiles x 16.
template <int DIM>
__global__ void __launch_bounds__(256) k_mlp_grad(const float *__restrict__ P, const double *__restrict__ st,
                                                  const double *__restrict__ T, int64_t count,
                                                  const int *__restrict__ idx, int64_t start, int64_t nbatch,
                                                  int tpw, float *__restrict__ partial, float *__restrict__ lossp) {
    __shared__ unsigned short sA[4][H][16];  // per wave: dz, neuron x sample (BF16)
    __shared__ unsigned short sB[4][H][16];  // per wave: activation, neuron x sample (BF16)
    __shared__ float red[kSurParams];        // block reduction
    __shared__ float lred[4];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const float *nrm = P + oNorm;
    const float inv_b = 2.0f / (float)nbatch;

    f32x4 dW3[4][4], dW2[4][4], dW1[4];
    float gb1[4][4], gb2[4][4], gb3[4][4], gW4[4][4];
    float gb4 = 0.0f, lsum = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        dW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            dW3[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            dW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            gb1[a][b] = gb2[a][b] = gb3[a][b] = gW4[a][b] = 0.0f;
        }
    }
    const int64_t spb = (int64_t)4 * tpw * 16;
    for (int t = 0; t < tpw; ++t) {
        const int64_t pos = (int64_t)blockIdx.x * spb + ((int64_t)w * tpw + t) * 16 + r;
        const bool valid = pos < nbatch;
        const int64_t n = valid ? (int64_t)idx[start + pos] : 0;
        float x[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float tgt = 0.0f;
        if (valid) {
            features<DIM>(st, count, n, nrm, x);
            tgt = (float)((T[n] - (double)nrm[12]) / (double)nrm[13]);
        }
        Fwd F;
        forward(P, x, r, g, F);
        const float res = valid ? (F.y + P[ob4] - tgt) : 0.0f;
        const float dy = inv_b * res;
        if (g == 0) {
            lsum = fmaf(res, res, lsum);
            gb4 += dy;
        }
        // output layer and dz3 (D layout)
        float dz[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * mt + 4 * g + j;
                gW4[mt][j] = fmaf(dy, F.h3[mt][j], gW4[mt][j]);
                dz[mt][j] = P[oW4 + k] * dy * (1.0f - F.h3[mt][j] * F.h3[mt][j]);
                gb3[mt][j] += dz[mt][j];
            }
        // ---- layer 3: dW3 += dz3 . h2^T ; dz2 = (W3^T dz3) * (1 - h2^2)
        for (int layer = 3; layer >= 1; --layer) {
            // stage dz (A) and the layer input (B) transposed through LDS
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 16 * mt + 4 * g + j;
                    sA[w][k][r] = to_bf16(dz[mt][j]);
                    if (layer == 3) sB[w][k][r] = to_bf16(F.h2[mt][j]);
                    if (layer == 2) sB[w][k][r] = to_bf16(F.h1[mt][j]);
                }
            if (layer == 1 && g == 0) {
#pragma unroll
                for (int k = 0; k < 16; ++k) sB[w][k][r] = k < 6 ? to_bf16(x[k]) : (unsigned short)0;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            bf16x4 Af[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                bf16x4 a;
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = (short)sA[w][16 * mt + r][4 * g + j];
                Af[mt] = a;
            }
            if (layer == 1) {
                bf16x4 b;
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = (short)sB[w][r][4 * g + j];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) dW1[mt] = mfma(Af[mt], b, dW1[mt]);
            } else {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    bf16x4 b;
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[j] = (short)sB[w][16 * nt + r][4 * g + j];
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) {
                        if (layer == 3) dW3[mt][nt] = mfma(Af[mt], b, dW3[mt][nt]);
                        else dW2[mt][nt] = mfma(Af[mt], b, dW2[mt][nt]);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (layer == 1) break;
            // back-propagate: dh = W^T dz (B operand = dz in D layout), dz_prev = dh * (1 - h^2)
            const float *Wl = layer == 3 ? P + oW3 : P + oW2;
            bf16x4 dzb[4];
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) dzb[kc] = pack4(dz[kc][0], dz[kc][1], dz[kc][2], dz[kc][3]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) acc = mfma(wtfrag(Wl, H, mt, kc, r, g), dzb[kc], acc);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float h = layer == 3 ? F.h2[mt][j] : F.h1[mt][j];
                    dz[mt][j] = acc[j] * (1.0f - h * h);
                    if (layer == 3) gb2[mt][j] += dz[mt][j];
                    else gb1[mt][j] += dz[mt][j];
                }
            }
        }
    }
    // sum the per-sample accumulators over the 16 sample lanes of each group
    auto rowsum = [](float v) {
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        return v;
    };
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            gb1[mt][j] = rowsum(gb1[mt][j]);
            gb2[mt][j] = rowsum(gb2[mt][j]);
            gb3[mt][j] = rowsum(gb3[mt][j]);
            gW4[mt][j] = rowsum(gW4[mt][j]);
        }
    gb4 = rowsum(gb4);
    lsum = rowsum(lsum);
    // deterministic block reduction: waves add in order 0..3
    for (int i = threadIdx.x; i < kSurParams; i += blockDim.x) red[i] = 0.0f;
    __syncthreads();
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 16 * mt + 4 * g + j;
                    if (r < kSurIn) red[oW1 + k * kSurIn + r] += dW1[mt][j];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        red[oW3 + k * H + 16 * nt + r] += dW3[mt][nt][j];
                        red[oW2 + k * H + 16 * nt + r] += dW2[mt][nt][j];
                    }
                    if (r == 0) {
                        red[ob1 + k] += gb1[mt][j];
                        red[ob2 + k] += gb2[mt][j];
                        red[ob3 + k] += gb3[mt][j];
                        red[oW4 + k] += gW4[mt][j];
                    }
                }
            }
            if (lane == 0) {
                red[ob4] += gb4;
                lred[ww] = lsum;
            }
        }
        __syncthreads();
    }
    float *out = partial + (size_t)blockIdx.x * kSurParams;
    for (int i = threadIdx.x; i < kSurParams; i += blockDim.x) out[i] = red[i];
    if (threadIdx.x == 0) lossp[blockIdx.x] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
}

// grad[i] = sum over blocks (in order) of partial[b][i]; loss accumulated.
__global__ void k_mlp_reduce(const float *__restrict__ partial, const float *__restrict__ lossp, int nblk,
                             float *__restrict__ grad, float *__restrict__ loss_acc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kSurParams) {
        float s = 0.0f;
        for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * kSurParams + i];
        grad[i] = s;
    }
    if (i == 0) {
        float l = 0.0f;
        for (int b = 0; b < nblk; ++b) l += lossp[b];
        loss_acc[0] += l;
    }
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kSurParams) return;
    const float gi = grad[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

int grid_for(int64_t count) {
    const int64_t waves = (count + 63) / 64;
    return (int)std::min<int64_t>((waves + 3) / 4, 2048);
}

}  // namespace

int surrogate_set(Surrogate &S, const float *host_params) {
    if (!S.params && hipMalloc(&S.params, (kSurParams + kSurNorm) * sizeof(float)) != hipSuccess) return -3;
    if (hipMemcpy(S.params, host_params, (kSurParams + kSurNorm) * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return -3;
    S.ready = true;
    return 0;
}

int surrogate_get(Surrogate &S, float *host_params) {
    return hipMemcpy(host_params, S.params, (kSurParams + kSurNorm) * sizeof(float), hipMemcpyDeviceToHost) ==
                   hipSuccess
               ? 0
               : -3;
}

int surrogate_predict(Surrogate &S, int dim, const double *states, int64_t count, double *Tg, hipStream_t s) {
    if (!S.ready) return -6;
    const int grid = grid_for(count);
    if (dim == 2) hipLaunchKernelGGL(k_mlp_predict<2>, dim3(grid), dim3(256), 0, s, S.params, states, count, Tg);
    else hipLaunchKernelGGL(k_mlp_predict<3>, dim3(grid), dim3(256), 0, s, S.params, states, count, Tg);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

static int ensure(float *&p, size_t n) {
    if (p) return 0;
    if (hipMalloc(&p, n * sizeof(float)) != hipSuccess) return -2;
    return hipMemset(p, 0, n * sizeof(float)) == hipSuccess ? 0 : -3;
}

// Gradient of the mean squared error over the samples idx[start .. start+nb)
// into S.grads; the summed squared residual is added to *loss_dev.
static int enqueue_grad(Surrogate &S, int dim, const double *states, const double *T, int64_t count, const int *idx,
                        int64_t start, int64_t nb, float *partial, float *lossp, float *loss_dev, int nblk_cap,
                        hipStream_t s) {
    const int tpw = 1;
    const int64_t spb = 4 * tpw * 16;
    const int nblk = (int)((nb + spb - 1) / spb);
    if (nblk > nblk_cap) return -1;
    if (dim == 2)
        hipLaunchKernelGGL(k_mlp_grad<2>, dim3(nblk), dim3(256), 0, s, S.params, states, T, count, idx, start, nb, tpw,
                           partial, lossp);
    else
        hipLaunchKernelGGL(k_mlp_grad<3>, dim3(nblk), dim3(256), 0, s, S.params, states, T, count, idx, start, nb, tpw,
                           partial, lossp);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kSurParams + 255) / 256), dim3(256), 0, s, partial, lossp, nblk, S.grads,
                       loss_dev);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int surrogate_grad(Surrogate &S, int dim, const double *states, const double *T, int64_t count, float *grad_host,
                   float *loss_host, hipStream_t s) {
    if (!S.ready) return -6;
    if (ensure(S.grads, kSurParams)) return -2;
    const int nblk = (int)((count + 63) / 64);
    float *partial = nullptr, *lossp = nullptr, *ld = nullptr;
    int *idx = nullptr;
    int rc = 0;
    std::vector<int> h(count);
    for (int64_t i = 0; i < count; ++i) h[i] = (int)i;
    if (hipMalloc(&partial, (size_t)nblk * kSurParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&lossp, nblk * sizeof(float)) != hipSuccess || hipMalloc(&ld, sizeof(float)) != hipSuccess ||
        hipMalloc(&idx, count * sizeof(int)) != hipSuccess)
        rc = -2;
    if (!rc && hipMemcpy(idx, h.data(), count * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) rc = -3;
    if (!rc && hipMemsetAsync(ld, 0, sizeof(float), s) != hipSuccess) rc = -3;
    if (!rc) rc = enqueue_grad(S, dim, states, T, count, idx, 0, count, partial, lossp, ld, nblk, s);
    if (!rc && hipMemcpyAsync(grad_host, S.grads, kSurParams * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = -3;
    float l = 0.0f;
    if (!rc && hipMemcpyAsync(&l, ld, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess) rc = -3;
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = -3;
    if (!rc && loss_host) *loss_host = l / (float)count;
    if (partial) (void)hipFree(partial);
    if (lossp) (void)hipFree(lossp);
    if (ld) (void)hipFree(ld);
    if (idx) (void)hipFree(idx);
    return rc;
}

int surrogate_train(Surrogate &S, int dim, const double *states, const double *T, int64_t count, int epochs, int batch,
                    float lr, uint64_t seed, float *loss_host, hipStream_t s) {
    if (!S.ready) {
        S.err = "set initial parameters (and normalisation) first";
        return -6;
    }
    if (ensure(S.grads, kSurParams) || ensure(S.adam_m, kSurParams) || ensure(S.adam_v, kSurParams)) return -2;
    const int nblk_cap = (batch + 63) / 64;
    float *partial = nullptr, *lossp = nullptr, *ld = nullptr;
    int *idx = nullptr;
    if (hipMalloc(&partial, (size_t)nblk_cap * kSurParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&lossp, nblk_cap * sizeof(float)) != hipSuccess || hipMalloc(&ld, sizeof(float)) != hipSuccess ||
        hipMalloc(&idx, count * sizeof(int)) != hipSuccess) {
        if (partial) (void)hipFree(partial);
        if (lossp) (void)hipFree(lossp);
        if (ld) (void)hipFree(ld);
        if (idx) (void)hipFree(idx);
        return -2;
    }
    std::vector<int> order(count);
    for (int64_t i = 0; i < count; ++i) order[i] = (int)i;
    std::mt19937_64 rng(seed);
    int rc = 0;
    // cosine learning-rate decay over this call's steps, lr -> 0
    const int64_t per_epoch = (count + batch - 1) / batch;
    const double total = (double)epochs * (double)per_epoch;
    int64_t t = 0;
    for (int ep = 0; ep < epochs && !rc; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        if (hipMemcpyAsync(idx, order.data(), count * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemsetAsync(ld, 0, sizeof(float), s) != hipSuccess) {
            rc = -3;
            break;
        }
        for (int64_t b0 = 0; b0 < count && !rc; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, count - b0);
            rc = enqueue_grad(S, dim, states, T, count, idx, b0, nb, partial, lossp, ld, nblk_cap, s);
            if (rc) break;
            ++S.step;
            const float c1 = 1.0f - std::pow(0.9f, (float)S.step);
            const float c2 = 1.0f - std::pow(0.999f, (float)S.step);
            const float lr_t = (float)(0.5 * lr * (1.0 + std::cos(3.14159265358979323846 * (double)t / total)));
            ++t;
            hipLaunchKernelGGL(k_adam, dim3((kSurParams + 255) / 256), dim3(256), 0, s, S.params, S.grads, S.adam_m,
                               S.adam_v, lr_t, c1, c2);
        }
        float l = 0.0f;
        if (!rc && (hipMemcpyAsync(&l, ld, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess))
            rc = -3;
        if (!rc && loss_host) loss_host[ep] = l / (float)count;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(partial);
    (void)hipFree(lossp);
    (void)hipFree(ld);
    (void)hipFree(idx);
    return rc;
}

// Normalisation (feature and temperature mean / standard deviation over the
// training set, host FP64) and Glorot-uniform initial weights from `seed`.
int surrogate_init(Surrogate &S, int dim, const double *states, const double *T, int64_t count, uint64_t seed,
                   hipStream_t s) {
    const int nvar = 5 + dim + 1;
    std::vector<double> h((size_t)nvar * count), ht(count);
    if (hipMemcpyAsync(h.data(), states, h.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(ht.data(), T, count * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return -3;
    double sum[7] = {0}, sq[7] = {0};
    for (int64_t i = 0; i < count; ++i) {
        double rho = 0.0, m2 = 0.0, f[7];
        for (int k = 0; k < 5; ++k) rho += h[k * count + i];
        for (int c = 0; c < dim; ++c) m2 += h[(5 + c) * count + i] * h[(5 + c) * count + i];
        for (int k = 0; k < 5; ++k) f[k] = std::log10(std::max(h[k * count + i], 1e-30));
        f[5] = (h[(5 + dim) * count + i] - 0.5 * m2 / rho) / rho;
        f[6] = ht[i];
        for (int k = 0; k < 7; ++k) {
            sum[k] += f[k];
            sq[k] += f[k] * f[k];
        }
    }
    std::vector<float> prm(kSurParams + kSurNorm, 0.0f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int rows, int cols) {
        const double lim = std::sqrt(6.0 / (rows + cols));
        std::uniform_real_distribution<double> U(-lim, lim);
        for (int i = 0; i < rows * cols; ++i) prm[off + i] = (float)U(rng);
    };
    fill(oW1, H, kSurIn);
    fill(oW2, H, H);
    fill(oW3, H, H);
    fill(oW4, 1, H);
    for (int k = 0; k < 7; ++k) {
        const double mean = sum[k] / count;
        const double var = std::max(sq[k] / count - mean * mean, 0.0);
        const double sd = std::sqrt(var) > 1e-12 * std::max(1.0, std::fabs(mean)) ? std::sqrt(var) : 1.0;
        if (k < 6) {
            prm[oNorm + k] = (float)mean;
            prm[oNorm + 6 + k] = (float)sd;
        } else {
            prm[oNorm + 12] = (float)mean;
            prm[oNorm + 13] = (float)sd;
        }
    }
    S.step = 0;
    if (S.adam_m) (void)hipMemset(S.adam_m, 0, kSurParams * sizeof(float));
    if (S.adam_v) (void)hipMemset(S.adam_v, 0, kSurParams * sizeof(float));
    return surrogate_set(S, prm.data());
}

void surrogate_free(Surrogate &S) {
    if (S.params) (void)hipFree(S.params);
    if (S.adam_m) (void)hipFree(S.adam_m);
    if (S.adam_v) (void)hipFree(S.adam_v);
    if (S.grads) (void)hipFree(S.grads);
    S = Surrogate();
}

}  // namespace dgx
