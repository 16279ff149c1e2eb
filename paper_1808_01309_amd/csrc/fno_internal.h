// Definitions shared by the neural-operator translation units: the operator's
// host state, BF16 rounding, GELU, and the fused inference kernels' entry
// points (one kernel per layer, see fno_fused.hip).
#pragma once
#include <math.h>

#include <string>

#include "fft_engine.h"
#include "plan.h"

typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace pst {

constexpr int GT = 256;  // threads per block of the FNO kernels

// FP32 -> BF16, round to nearest even (inputs are finite)
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.  erf from the rational
// approximation of Abramowitz & Stegun (Handbook of Mathematical Functions,
// eq. 7.1.26, |error| <= 1.5e-7 on z >= 0):
//   1 - erf(z) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-z^2),  t = 1 / (1 + p z),
// evaluated branch-free with the hardware reciprocal and exponential; 1 + erf
// is formed without cancellation for x < 0.  About a third of the
// instructions of the library erff, far below FP32 parity tolerances.
__device__ __forceinline__ float gelu_f(float x) {
    const float z = fabsf(x) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, z, 1.0f));
    float q = fmaf(t, 1.061405429f, -1.453152027f);
    q = fmaf(t, q, 1.421413741f);
    q = fmaf(t, q, -0.284496736f);
    q = fmaf(t, q, 0.254829592f);
    const float c = q * t * __expf(-z * z);  // 1 - erf(|x| / sqrt 2)
    return 0.5f * x * (x < 0.f ? c : 2.0f - c);
}
// derivative of the exact-erf GELU (training)
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

}  // namespace pst

// A dense (pointwise) layer W [O][K] + b: offsets into the parameter vector and
// padded BF16 / FP32 copies of W and of its transpose.
struct FnoDense {
    int O, K, Opad, Kpad, To, Tk;   // To x Tk: transposed padded shape
    int64_t off;                    // offset of W in theta (bias follows at off + O K)
    unsigned short *Wb, *Tb;
    float *Wf, *Tf;
};

struct pst_fno {
    pst_fno_params p;
    hipStream_t stream;
    pst_plan* fft;            // transform plan of size n (its FFT kernels)
    int P, nxh, nm;
    int64_t fsz, nparam;
    float *theta, *grad, *am, *av;
    int64_t adam_t;
    FnoDense lift, wc[8], q1, q2;
    int64_t offR[8];
    int *modeoff;
    float* modew;
    float *v, *s, *kb, *pre, *out, *dv, *ds, *dpre, *dout, *tmp;
    pst::cx<float> *specA, *specB, *ffttmp, *vst;
    void* fact;               // fused inference activations: two slots of fact_slot bytes
    int64_t fact_slot;
    float* part;
    double* lpart;
    float* coef;
    int64_t wpart_floats;
    std::string msg;
};

namespace pst {

// Channel stride of the fused inference activations ([b][point][channel]):
// BF16 rows padded to whole 16-channel MFMA K steps, FP32 rows unpadded.
__host__ __device__ constexpr int fno_act_cp(int W, bool bf) { return bf ? (W + 15) / 16 * 16 : W; }

// Fused inference kernels (grid sizes n with an instantiation; false otherwise).
// Activations between layers ([b][point][channel], channel stride fno_act_cp)
// are BF16 when the operator runs on the matrix cores, FP32 otherwise; t1 holds
// the x-transformed lines [b][c][z][y][kx < m].
bool fno_fused_supported(int n);
//   v0 = lift(u) -> act, x r2c of v0 -> t1
void fno_fused_lift(pst_fno* F, const float* u, int B, void* act, cx<float>* t1);
//   s = Wc_l v_l + b_l + x c2r(t1); v_{l+1} = gelu(s) -> act_out, x r2c(v_{l+1}) -> t1 (in place)
void fno_fused_layer(pst_fno* F, int l, int B, const void* act_in, void* act_out, cx<float>* t1);
//   last layer (no activation) and projection: out = u + Wq2 gelu(Wq1 v_L + bq1) + bq2
void fno_fused_last(pst_fno* F, int l, int B, const void* act_in, cx<float>* t1, const float* u, float* out);

}  // namespace pst
