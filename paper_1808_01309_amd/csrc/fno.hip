// Fourier neural operator surrogate: forward, loss, backward and Adam, all in
// hand-written HIP for gfx950.
//
//   v0 = Wl u + bl;  s_l = Wc_l v_l + bc_l + K_l(v_l);  v_{l+1} = gelu(s_l)
//   (identity after the last layer);  out = u + Wq2 gelu(Wq1 v_L + bq1) + bq2,
//   K_l(v) = c2r(R_l . r2c(v) on the retained modes).
//
// Channel mixing (every dense layer, forward and backward) is a GEMM over
// points on the matrix cores: gfx950's v_mfma_f32_32x32x16_bf16 with BF16
// weights and activations and FP32 accumulation (an FP32 FMA variant of the same kernels
// exists for gradient checks).  The spectral layers run the library's own 3D
// r2c / c2r transform kernels; the per-mode complex channel mixing and its
// adjoint are FP32.  Activations are stored FP32, channel-major
// [batch][channel][n^3].
//
// Adjoints (weighted inner product on half spectra, weight w = 1 on kx = 0,
// else 2): c2r^T = n^3 r2c, r2c^T = c2r / n^3.  With S = r2c(ds) (scaled by
// 1/n^3): g_R = n^3 w S conj(V),  g_v = c2r(conj(R)^T S).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "fno_internal.h"

using namespace pst;

namespace {

enum { EPI_NONE = 0, EPI_GELU = 1, EPI_DGELU = 2 };

// out[b][o][p] = epi( sum_k W[o][k] X'[b][k][p] + bias[o] + add[b][o][p] ),
// X' = gelu(X) if GELU_IN.  One wave computes 32 points x 32 output channels
// (output tile blockIdx.y); the K loop steps by 16 (one MFMA, gfx950's
// 32x32x16 BF16 form; Kpad is a multiple of 16).
//   MFMA operands: A[m][k] lane m + 32 ((k / 8) % 2), element k % 8 of step
//   k / 16; B[k][n] lane n + 32 ((k / 8) % 2); D[m][n] lane n + 32 ((m / 4) % 2),
//   register (m % 4) + 4 (m / 8).
template <bool MFMA, bool GELU_IN, int EPI>
__global__ __launch_bounds__(GT) void k_gemm(const unsigned short* __restrict__ Wb, const float* __restrict__ Wf,
                                             int Kpad, int K, int O, const float* __restrict__ X,
                                             const float* __restrict__ bias, const float* __restrict__ add,
                                             const float* __restrict__ aux, float* __restrict__ pre,
                                             float* __restrict__ out, int P, int64_t total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t gp0 = ((int64_t)blockIdx.x * (GT / 64) + wave) * 32;
    if (gp0 >= total) return;  // no block-level synchronisation below
    const int b = (int)(gp0 / P), p0 = (int)(gp0 % P);
    const int n = lane & 31, kg = lane >> 5;
    const int ot = blockIdx.y;
    const float* Xb = X + (int64_t)b * K * P + p0 + n;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    if constexpr (MFMA) {
        const unsigned short* wrow = Wb + (int64_t)(ot * 32 + n) * Kpad + 8 * kg;
        for (int s = 0; s < Kpad / 16; ++s) {
            bf16x8v bb;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 16 * s + 8 * kg + j;
                float x = k < K ? Xb[(int64_t)k * P] : 0.f;
                if (GELU_IN) x = gelu_f(x);
                bb[j] = (__bf16)x;
            }
            const bf16x8v aa = *(const bf16x8v*)(wrow + 16 * s);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aa, bb, acc, 0, 0, 0);
        }
    } else {
        for (int k = 0; k < K; ++k) {
            float x = Xb[(int64_t)k * P];
            if (GELU_IN) x = gelu_f(x);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = 8 * (r / 4) + 4 * kg + (r % 4);
                acc[r] += Wf[(int64_t)(ot * 32 + m) * Kpad + k] * x;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int o = ot * 32 + 8 * (r / 4) + 4 * kg + (r % 4);
        if (o >= O) continue;
        const int64_t idx = ((int64_t)b * O + o) * P + p0 + n;
        float s = acc[r];
        if (bias) s += bias[o];
        if (add) s += add[idx];
        if (EPI == EPI_GELU) {
            pre[idx] = s;
            out[idx] = gelu_f(s);
        } else if (EPI == EPI_DGELU) {
            out[idx] = s * gelu_grad_f(aux[idx]);
        } else {
            out[idx] = s;
        }
    }
}

// Partial weight gradients: dW[o][k] = sum_{b,p} Y[b][o][p] X'[b][k][p] over
// this block's points (16 per MFMA step), tile (ot, kt) = blockIdx.y.
template <bool MFMA, bool GELU_X>
__global__ __launch_bounds__(GT) void k_wgrad(const float* __restrict__ Y, int O, const float* __restrict__ X, int K,
                                              int P, int64_t total, int64_t ppb, int ktiles,
                                              float* __restrict__ partial) {
    __shared__ float red[GT / 64][16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 31, kg = lane >> 5;
    const int ot = blockIdx.y / ktiles, kt = blockIdx.y % ktiles;
    const int om = ot * 32 + n, kn = kt * 32 + n;  // A row (as m) and B column (as n) of this lane
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    // points per step: 16 (one 32x32x16 MFMA) or 8; P and the block ranges are multiples of 16
    constexpr int PS = MFMA ? 16 : 8;
    const int64_t beg = (int64_t)blockIdx.x * ppb, end = beg + ppb < total ? beg + ppb : total;
    for (int64_t q = beg + (int64_t)wave * PS; q < end; q += PS * (GT / 64)) {
        const int b = (int)(q / P), p = (int)(q % P);
        if constexpr (MFMA) {
            // lane n + 32 kg: points p + 8 kg .. + 7 of row om (A) and column kn (B)
            bf16x8v aa, bb;
            const float* yr = Y + ((int64_t)b * O + om) * P + p + 8 * kg;
            const float* xr = X + ((int64_t)b * K + kn) * P + p + 8 * kg;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float4 ya = om < O ? *(const float4*)(yr + 4 * h) : make_float4(0, 0, 0, 0);
                float4 xb = kn < K ? *(const float4*)(xr + 4 * h) : make_float4(0, 0, 0, 0);
                if (GELU_X && kn < K) {
                    xb.x = gelu_f(xb.x); xb.y = gelu_f(xb.y); xb.z = gelu_f(xb.z); xb.w = gelu_f(xb.w);
                }
                aa[4 * h] = (__bf16)ya.x; aa[4 * h + 1] = (__bf16)ya.y; aa[4 * h + 2] = (__bf16)ya.z; aa[4 * h + 3] = (__bf16)ya.w;
                bb[4 * h] = (__bf16)xb.x; bb[4 * h + 1] = (__bf16)xb.y; bb[4 * h + 2] = (__bf16)xb.z; bb[4 * h + 3] = (__bf16)xb.w;
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aa, bb, acc, 0, 0, 0);
        } else {
            for (int j = 0; j < 8; ++j) {
                float x = kn < K ? X[((int64_t)b * K + kn) * P + p + j] : 0.f;
                if (GELU_X) x = gelu_f(x);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int o = ot * 32 + 8 * (r / 4) + 4 * kg + (r % 4);
                    const float y = o < O ? Y[((int64_t)b * O + o) * P + p + j] : 0.f;
                    acc[r] += y * x;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
    __syncthreads();
    // lane-ordered sum over the waves, written as [m][n] of the 32 x 32 tile
    for (int i = threadIdx.x; i < 16 * 64; i += GT) {
        const int r = i / 64, l = i % 64;
        float s = 0.f;
        for (int w = 0; w < GT / 64; ++w) s += red[w][r][l];
        const int m = 8 * (r / 4) + 4 * (l >> 5) + (r % 4), nn = l & 31;
        partial[((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * 1024 + m * 32 + nn] = s;
    }
}

// dW = sum of the block partials (fixed order) into grad[off + o K + k]
__global__ void k_wgrad_reduce(const float* __restrict__ partial, int nblk, int ntiles, int ktiles, int O, int K,
                               float* __restrict__ grad) {
    const int t = blockIdx.x;
    const int ot = t / ktiles, kt = t % ktiles;
    // one thread per tile element (blockIdx.y selects 64 of the 1024)
    for (int i = blockIdx.y * blockDim.x + threadIdx.x; i < 1024; i += gridDim.y * blockDim.x) {
        const int m = i / 32, nn = i % 32;
        const int o = ot * 32 + m, k = kt * 32 + nn;
        if (o >= O || k >= K) continue;
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += partial[((int64_t)b * ntiles + t) * 1024 + i];
        grad[o * K + k] = (float)s;
    }
}

// db[o] = sum_{b,p} Y[b][o][p] in two fixed-order levels: block (o, c) sums
// the point range c of every batch item (FP64, tree over the block), then one
// thread per channel adds the BG_CHUNKS partials in order.
constexpr int BG_CHUNKS = 64;
__global__ __launch_bounds__(GT) void k_bgrad_part(const float* __restrict__ Y, int O, int P, int B,
                                                   double* __restrict__ part) {
    __shared__ double sh[GT];
    const int o = blockIdx.x, c = blockIdx.y;
    const int len = (P + BG_CHUNKS - 1) / BG_CHUNKS;
    const int p0 = c * len, p1 = p0 + len < P ? p0 + len : P;
    double s = 0.0;
    for (int b = 0; b < B; ++b) {
        const float* y = Y + ((int64_t)b * O + o) * P;
        for (int p = p0 + threadIdx.x; p < p1; p += GT) s += y[p];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = GT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[o * BG_CHUNKS + c] = sh[0];
}
__global__ void k_bgrad_reduce(const double* __restrict__ part, int O, float* __restrict__ grad) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    double s = 0.0;
    for (int c = 0; c < BG_CHUNKS; ++c) s += part[o * BG_CHUNKS + c];
    grad[o] = (float)s;
}

// forward spectral mixing on compact spectra [b][c][mode] (mode stride 1,
// channel stride nm): out[b][o][m] = sum_c R[m][c][o] V[b][c][m].  A block
// takes MB consecutive modes so that every (b, c) row is read and written as
// one contiguous MB-element segment; the modes' slices meet in LDS.  A thread
// owns one (mode, o) and accumulates 8 batch entries at a time: the weights
// R[m][c][o] are read straight from memory (consecutive o in consecutive
// lanes), the spectra from LDS (the lanes of a wavefront read a few addresses:
// broadcasts).
//   LDS: Vh [MB][B C], Out [MB][B O]
__global__ __launch_bounds__(GT) void k_mix_fwd(const cx<float>* __restrict__ spec_in, const cx<float>* __restrict__ R,
                                                int nm, int MB, int B, int C, int O, cx<float>* __restrict__ spec_out,
                                                cx<float>* __restrict__ vstore) {
    extern __shared__ cx<float> shm[];
    cx<float>* Vh = shm;
    cx<float>* Out = Vh + MB * B * C;
    const int m0 = blockIdx.x * MB;
    const int mb = nm - m0 < MB ? nm - m0 : MB;
    for (int q = threadIdx.x; q < B * C * MB; q += GT) {
        const int i = q / MB, mm = q % MB;
        if (mm >= mb) continue;
        const cx<float> v = spec_in[(int64_t)i * nm + m0 + mm];
        Vh[mm * B * C + i] = v;
        if (vstore) vstore[(int64_t)(m0 + mm) * B * C + i] = v;
    }
    __syncthreads();
    constexpr int BB = 8;
    for (int t = threadIdx.x; t < mb * O; t += GT) {
        const int mm = t / O, o = t % O;
        const cx<float>* Rm = R + (int64_t)(m0 + mm) * C * O + o;
        const cx<float>* V = Vh + mm * B * C;
        for (int b0 = 0; b0 < B; b0 += BB) {
            cx<float> acc[BB];
#pragma unroll
            for (int bb = 0; bb < BB; ++bb) acc[bb] = czero<float>();
#pragma unroll 8
            for (int c = 0; c < C; ++c) {
                const cx<float> r = Rm[(int64_t)c * O];
#pragma unroll
                for (int bb = 0; bb < BB; ++bb) {
                    if (b0 + bb >= B) break;
                    const cx<float> v = V[(b0 + bb) * C + c];
                    acc[bb].x += r.x * v.x - r.y * v.y;
                    acc[bb].y += r.x * v.y + r.y * v.x;
                }
            }
#pragma unroll
            for (int bb = 0; bb < BB; ++bb)
                if (b0 + bb < B) Out[mm * B * O + (b0 + bb) * O + o] = acc[bb];
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < B * O * MB; q += GT) {
        const int i = q / MB, mm = q % MB;
        if (mm < mb) spec_out[(int64_t)i * nm + m0 + mm] = Out[mm * B * O + i];
    }
}

// adjoint spectral mixing: S = r2c(ds) at the mode (scaled 1/n^3)
//   g_v(mode) = sum_o conj(R[c][o]) S[b][o]          (into spec_out for c2r)
//   g_R[c][o] = n^3 w(mode) sum_b S[b][o] conj(V[b][c])
__global__ __launch_bounds__(GT) void k_mix_bwd(const cx<float>* __restrict__ spec_g, const cx<float>* __restrict__ R,
                                                const cx<float>* __restrict__ vstore, const int* __restrict__ modeoff,
                                                const float* __restrict__ modew, int64_t fsz, int B, int C, int O,
                                                float P3, cx<float>* __restrict__ spec_out, cx<float>* __restrict__ gR) {
    extern __shared__ cx<float> shm[];
    cx<float>* S = shm;                  // [B][O]
    cx<float>* Vh = shm + B * O;         // [B][C]
    cx<float>* Rm = Vh + B * C;          // [C][O]
    const int m = blockIdx.x;
    const int64_t off = modeoff[m];
    for (int i = threadIdx.x; i < B * O; i += GT) S[i] = spec_g[(int64_t)i * fsz + off];
    for (int i = threadIdx.x; i < B * C; i += GT) Vh[i] = vstore[(int64_t)m * B * C + i];
    for (int i = threadIdx.x; i < C * O; i += GT) Rm[i] = R[(int64_t)m * C * O + i];
    __syncthreads();
    for (int i = threadIdx.x; i < B * C; i += GT) {
        const int b = i / C, c = i % C;
        float re = 0.f, im = 0.f;
        for (int o = 0; o < O; ++o) {
            const cx<float> r = Rm[c * O + o], s = S[b * O + o];
            re += r.x * s.x + r.y * s.y;   // conj(r) s
            im += r.x * s.y - r.y * s.x;
        }
        spec_out[(int64_t)i * fsz + off] = {re, im};
    }
    const float scale = P3 * modew[m];
    for (int i = threadIdx.x; i < C * O; i += GT) {
        const int c = i / O, o = i % O;
        float re = 0.f, im = 0.f;
        for (int b = 0; b < B; ++b) {
            const cx<float> s = S[b * O + o], v = Vh[b * C + c];
            re += s.x * v.x + s.y * v.y;   // s conj(v)
            im += s.y * v.x - s.x * v.y;
        }
        gR[(int64_t)m * C * O + i] = {scale * re, scale * im};
    }
}

__global__ void k_fill0(float* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.f;
}

__global__ void k_add(float* __restrict__ a, const float* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] += b[i];
}

// ds = dv * gelu'(s)
__global__ void k_dgelu(const float* __restrict__ dv, const float* __restrict__ s, float* __restrict__ ds, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        ds[i] = dv[i] * gelu_grad_f(s[i]);
}

// per-sample sums of (out - tgt)^2 and tgt^2 (block partials, double)
__global__ __launch_bounds__(GT) void k_loss_part(const float* __restrict__ out, const float* __restrict__ tgt,
                                                  int64_t per, double* __restrict__ part) {
    __shared__ double se[GT], st[GT];
    const int b = blockIdx.y;
    double e2 = 0.0, t2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < per; i += (int64_t)gridDim.x * GT) {
        const double t = tgt[b * per + i], e = out[b * per + i] - t;
        e2 += e * e;
        t2 += t * t;
    }
    se[threadIdx.x] = e2;
    st[threadIdx.x] = t2;
    __syncthreads();
    for (int w = GT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            se[threadIdx.x] += se[threadIdx.x + w];
            st[threadIdx.x] += st[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((int64_t)b * gridDim.x + blockIdx.x) * 2] = se[0];
        part[((int64_t)b * gridDim.x + blockIdx.x) * 2 + 1] = st[0];
    }
}

__global__ void k_loss_grad(const float* __restrict__ out, const float* __restrict__ tgt, const float* __restrict__ coef,
                            int64_t per, int B, float* __restrict__ dout) {
    const int64_t n = per * B;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dout[i] = (out[i] - tgt[i]) * coef[i / per];
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// padded copies of a dense weight [O][K] (at theta + off): W [Opad][Kpad] and
// its transpose WT [Kpad'][Opad'] (Kpad' = roundup(K, 32), Opad' = roundup(O, 16)),
// both as BF16 and FP32
__global__ void k_pack(const float* __restrict__ w, int O, int K, int Opad, int Kpad, int Tpad_o, int Tpad_k,
                       unsigned short* __restrict__ Wb, float* __restrict__ Wf, unsigned short* __restrict__ Tb,
                       float* __restrict__ Tf) {
    const int n1 = Opad * Kpad, n2 = Tpad_o * Tpad_k;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2; i += gridDim.x * blockDim.x) {
        if (i < n1) {
            const int o = i / Kpad, k = i % Kpad;
            const float x = (o < O && k < K) ? w[o * K + k] : 0.f;
            Wb[i] = f2bf(x);
            Wf[i] = x;
        } else {
            const int j = i - n1;
            const int k = j / Tpad_k, o = j % Tpad_k;  // WT[k][o] = W[o][k]
            const float x = (o < O && k < K) ? w[o * K + k] : 0.f;
            Tb[j] = f2bf(x);
            Tf[j] = x;
        }
    }
}

unsigned gs(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

// =================================================================== host side
static thread_local std::string g_fno_err;

static pst_status ffail(pst_fno* F, pst_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (F) F->msg = buf;
    else g_fno_err = buf;
    return s;
}

static int rup(int a, int b) { return (a + b - 1) / b * b; }

extern "C" const char* pst_fno_last_error(const pst_fno* F) { return F ? F->msg.c_str() : g_fno_err.c_str(); }

extern "C" void pst_fno_destroy(pst_fno* F) {
    if (!F) return;
    hipStreamSynchronize(F->stream);
    std::vector<void*> bufs = {F->theta, F->grad, F->am, F->av, F->modeoff, F->modew, F->v, F->s, F->kb, F->pre,
                               F->out, F->dv, F->ds, F->dpre, F->dout, F->tmp, F->specA, F->specB, F->ffttmp,
                               F->vst, F->part, F->lpart, F->coef, F->fact};
    FnoDense* ds[] = {&F->lift, &F->q1, &F->q2};
    for (FnoDense* d : ds)
        for (void* b : {(void*)d->Wb, (void*)d->Tb, (void*)d->Wf, (void*)d->Tf}) bufs.push_back(b);
    for (int l = 0; l < F->p.layers; ++l)
        for (void* b : {(void*)F->wc[l].Wb, (void*)F->wc[l].Tb, (void*)F->wc[l].Wf, (void*)F->wc[l].Tf}) bufs.push_back(b);
    for (void* b : bufs)
        if (b) hipFree(b);
    if (F->fft) pst_plan_destroy(F->fft);
    delete F;
}

static bool dmalloc(void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return false;
    }
    return true;
}

static bool make_dense(FnoDense& d, int O, int K, int64_t off) {
    d.O = O;
    d.K = K;
    d.Opad = rup(O, 32);
    d.Kpad = rup(K, 16);
    d.To = rup(K, 32);
    d.Tk = rup(O, 16);
    d.off = off;
    return dmalloc((void**)&d.Wb, sizeof(unsigned short) * d.Opad * d.Kpad) &&
           dmalloc((void**)&d.Wf, sizeof(float) * d.Opad * d.Kpad) &&
           dmalloc((void**)&d.Tb, sizeof(unsigned short) * d.To * d.Tk) &&
           dmalloc((void**)&d.Tf, sizeof(float) * d.To * d.Tk);
}

static void pack(pst_fno* F, FnoDense& d) {
    hipLaunchKernelGGL(k_pack, dim3(gs(d.Opad * d.Kpad + d.To * d.Tk)), dim3(256), 0, F->stream, F->theta + d.off, d.O,
                       d.K, d.Opad, d.Kpad, d.To, d.Tk, d.Wb, d.Wf, d.Tb, d.Tf);
}

static void pack_all(pst_fno* F) {
    pack(F, F->lift);
    for (int l = 0; l < F->p.layers; ++l) pack(F, F->wc[l]);
    pack(F, F->q1);
    pack(F, F->q2);
}

extern "C" pst_status pst_fno_create(const pst_fno_params* p, void* hip_stream, pst_fno** out) {
    g_fno_err.clear();
    if (!out || !p) return ffail(nullptr, PST_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (!pst_supported_n(p->n)) return ffail(nullptr, PST_ERR_UNSUPPORTED_N, "n = %d", p->n);
    if (p->width < 1 || p->width > 64 || p->modes < 1 || 2 * p->modes > p->n || p->layers < 1 || p->layers > 8 ||
        p->hidden < 1 || p->hidden > 256 || p->batch < 1 || p->batch > 64)
        return ffail(nullptr, PST_ERR_INVALID_ARG, "width 1..64, 1 <= modes <= n/2, layers 1..8, hidden 1..256, batch 1..64");
    if (2 * p->batch * p->width + p->width * p->width > 8192)
        return ffail(nullptr, PST_ERR_INVALID_ARG, "2 batch width + width^2 must not exceed 8192 (spectral mixing LDS)");
    if ((long)p->n * p->n * p->n % 32 != 0) return ffail(nullptr, PST_ERR_UNSUPPORTED_N, "n^3 must be a multiple of 32");
    pst_fno* F = new pst_fno();
    F->p = *p;
    F->stream = (hipStream_t)hip_stream;
    const int n = p->n, W = p->width, m = p->modes, L = p->layers, H = p->hidden, B = p->batch;
    F->P = n * n * n;
    F->nxh = n / 2 + 1;
    F->nm = 4 * m * m * m;
    F->fsz = F->nm;  // compact spectra [batch][channel][mode]
    pst_params fp{n, PST_NS, PST_FP32, 4, 0.0, 0.0, 1.0, PST_DEALIAS_CUBE, 0};
    if (pst_plan_create(&fp, hip_stream, &F->fft) != PST_OK) {
        g_fno_err = std::string("transform plan: ") + pst_last_error(nullptr);
        delete F;
        return PST_ERR_HIP;
    }
    // parameter layout (matches the oracle): Wl, bl, {Wc, bc, R}*, Wq1, bq1, Wq2, bq2
    int64_t off = 0;
    bool ok = make_dense(F->lift, W, 3, off);
    off += W * 3 + W;
    for (int l = 0; l < L; ++l) {
        ok = ok && make_dense(F->wc[l], W, W, off);
        off += W * W + W;
        F->offR[l] = off;
        off += (int64_t)F->nm * W * W * 2;
    }
    ok = ok && make_dense(F->q1, H, W, off);
    off += H * W + H;
    ok = ok && make_dense(F->q2, 3, H, off);
    off += 3 * H + 3;
    F->nparam = off;
    const int64_t act = (int64_t)B * W * F->P, pre = (int64_t)B * H * F->P, io = (int64_t)B * 3 * F->P;
    const int64_t spec = (int64_t)B * W * F->nm;
    const int64_t wsp = (int64_t)B * W * n * n * m + (int64_t)B * W * n * 2 * m * m;  // pruned-transform workspace
    F->wpart_floats = (int64_t)1024 * 16 * 1024;  // blocks x tiles x 32 x 32 (upper bound used below)
    ok = ok && dmalloc((void**)&F->theta, 4 * off) && dmalloc((void**)&F->grad, 4 * off) &&
         dmalloc((void**)&F->am, 4 * off) && dmalloc((void**)&F->av, 4 * off) &&
         dmalloc((void**)&F->modeoff, sizeof(int) * F->nm) && dmalloc((void**)&F->modew, sizeof(float) * F->nm) &&
         dmalloc((void**)&F->v, 4 * act * (L + 1)) && dmalloc((void**)&F->s, 4 * act * L) &&
         dmalloc((void**)&F->kb, 4 * act) && dmalloc((void**)&F->pre, 4 * pre) && dmalloc((void**)&F->out, 4 * io) &&
         dmalloc((void**)&F->dv, 4 * act) && dmalloc((void**)&F->ds, 4 * act) && dmalloc((void**)&F->dpre, 4 * pre) &&
         dmalloc((void**)&F->dout, 4 * io) && dmalloc((void**)&F->tmp, 4 * act) &&
         dmalloc((void**)&F->specA, 8 * spec) && dmalloc((void**)&F->specB, 8 * spec) &&
         dmalloc((void**)&F->ffttmp, 8 * wsp) && dmalloc((void**)&F->vst, 8 * (int64_t)L * F->nm * B * W) &&
         dmalloc((void**)&F->part, 4 * F->wpart_floats) && dmalloc((void**)&F->lpart, sizeof(double) * 2 * 64 * 1024) &&
         dmalloc((void**)&F->coef, sizeof(float) * 64);
    // fused inference activations: two slots, point-major with the padded channel stride
    F->fact_slot = (int64_t)B * F->P * fno_act_cp(W, p->mfma != 0) * (p->mfma ? 2 : 4);
    F->fact_slot = (F->fact_slot + 255) / 256 * 256;
    ok = ok && (!fno_fused_supported(n) || dmalloc(&F->fact, 2 * (size_t)F->fact_slot));
    if (!ok) {
        g_fno_err = "device allocation failed";
        pst_fno_destroy(F);
        return PST_ERR_OOM;
    }
    // retained modes, in the order the pruned transforms produce them: kx fastest
    // in [0, m), then ky, then kz, each in [0, m) U [n - m, n); the offset of a
    // mode in a compact spectrum is its index.  Weight 1 on the kx = 0 plane
    // (m <= n/2 keeps the Nyquist plane out), 2 elsewhere.
    std::vector<int> mo(F->nm);
    std::vector<float> mw(F->nm);
    for (int i = 0; i < F->nm; ++i) {
        mo[i] = i;
        mw[i] = (i % m == 0) ? 1.f : 2.f;
    }
    hipMemcpy(F->modeoff, mo.data(), sizeof(int) * F->nm, hipMemcpyHostToDevice);
    hipMemcpy(F->modew, mw.data(), sizeof(float) * F->nm, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(k_fill0, dim3(gs(off)), dim3(256), 0, F->stream, F->theta, off);
    hipLaunchKernelGGL(k_fill0, dim3(gs(off)), dim3(256), 0, F->stream, F->am, off);
    hipLaunchKernelGGL(k_fill0, dim3(gs(off)), dim3(256), 0, F->stream, F->av, off);
    pack_all(F);
    if (hipStreamSynchronize(F->stream) != hipSuccess) {
        g_fno_err = "initialisation failed";
        pst_fno_destroy(F);
        return PST_ERR_HIP;
    }
    *out = F;
    return PST_OK;
}

extern "C" pst_status pst_fno_param_count(const pst_fno* F, long long* count) {
    if (!F || !count) return PST_ERR_INVALID_ARG;
    *count = F->nparam;
    return PST_OK;
}

extern "C" pst_status pst_fno_set_params(pst_fno* F, const float* theta, int mem) {
    if (!F || !theta) return PST_ERR_INVALID_ARG;
    if (hipMemcpyAsync(F->theta, theta, 4 * F->nparam, mem == PST_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                       F->stream) != hipSuccess)
        return ffail(F, PST_ERR_HIP, "parameter copy failed");
    pack_all(F);
    F->adam_t = 0;
    hipLaunchKernelGGL(k_fill0, dim3(gs(F->nparam)), dim3(256), 0, F->stream, F->am, F->nparam);
    hipLaunchKernelGGL(k_fill0, dim3(gs(F->nparam)), dim3(256), 0, F->stream, F->av, F->nparam);
    if (mem == PST_MEM_HOST && hipStreamSynchronize(F->stream) != hipSuccess) return ffail(F, PST_ERR_HIP, "sync failed");
    return PST_OK;
}

static pst_status copy_out(pst_fno* F, const float* src, float* dst, int mem) {
    if (!dst) return ffail(F, PST_ERR_INVALID_ARG, "NULL output");
    if (hipMemcpyAsync(dst, src, 4 * F->nparam, mem == PST_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                       F->stream) != hipSuccess ||
        (mem == PST_MEM_HOST && hipStreamSynchronize(F->stream) != hipSuccess))
        return ffail(F, PST_ERR_HIP, "copy failed");
    return PST_OK;
}

extern "C" pst_status pst_fno_get_params(pst_fno* F, float* theta, int mem) {
    if (!F) return PST_ERR_INVALID_ARG;
    return copy_out(F, F->theta, theta, mem);
}

extern "C" pst_status pst_fno_get_grad(pst_fno* F, float* grad, int mem) {
    if (!F) return PST_ERR_INVALID_ARG;
    return copy_out(F, F->grad, grad, mem);
}

// dense layer: out = epi(W X' + b + add)
static void dense_fwd(pst_fno* F, const FnoDense& d, bool transposed, const float* X, int B, const float* bias,
                      const float* add, const float* aux, float* pre, float* out, int epi, bool gelu_in) {
    const int O = transposed ? d.K : d.O, K = transposed ? d.O : d.K;
    const int Kpad = transposed ? d.Tk : d.Kpad, Opad = transposed ? d.To : d.Opad;
    const unsigned short* Wb = transposed ? d.Tb : d.Wb;
    const float* Wf = transposed ? d.Tf : d.Wf;
    const int64_t total = (int64_t)B * F->P;
    dim3 grid((unsigned)((total + 127) / 128), Opad / 32);
#define GEMM_LAUNCH(M, G, E)                                                                                      \
    hipLaunchKernelGGL((k_gemm<M, G, E>), grid, dim3(GT), 0, F->stream, Wb, Wf, Kpad, K, O, X, bias, add, aux, pre, \
                       out, F->P, total)
    const bool mf = F->p.mfma != 0;
    if (mf) {
        if (gelu_in) GEMM_LAUNCH(true, true, EPI_NONE);
        else if (epi == EPI_GELU) GEMM_LAUNCH(true, false, EPI_GELU);
        else if (epi == EPI_DGELU) GEMM_LAUNCH(true, false, EPI_DGELU);
        else GEMM_LAUNCH(true, false, EPI_NONE);
    } else {
        if (gelu_in) GEMM_LAUNCH(false, true, EPI_NONE);
        else if (epi == EPI_GELU) GEMM_LAUNCH(false, false, EPI_GELU);
        else if (epi == EPI_DGELU) GEMM_LAUNCH(false, false, EPI_DGELU);
        else GEMM_LAUNCH(false, false, EPI_NONE);
    }
#undef GEMM_LAUNCH
}

// weight and bias gradients of a dense layer: dW = Y X'^T, db = sum Y
static void dense_grad(pst_fno* F, const FnoDense& d, const float* Y, const float* X, int B, bool gelu_x) {
    const int64_t total = (int64_t)B * F->P;
    const int otiles = d.Opad / 32, ktiles = rup(d.K, 32) / 32, ntiles = otiles * ktiles;
    int nblk = (int)((total + 8191) / 8192);
    const int maxblk = (int)(F->wpart_floats / (1024 * (int64_t)ntiles));
    if (nblk > maxblk) nblk = maxblk;
    if (nblk < 1) nblk = 1;
    const int64_t ppb = ((total + nblk - 1) / nblk + 31) / 32 * 32;
    nblk = (int)((total + ppb - 1) / ppb);
    dim3 grid(nblk, ntiles);
    const bool mf = F->p.mfma != 0;
    if (mf && gelu_x)
        hipLaunchKernelGGL((k_wgrad<true, true>), grid, dim3(GT), 0, F->stream, Y, d.O, X, d.K, F->P, total, ppb, ktiles, F->part);
    else if (mf)
        hipLaunchKernelGGL((k_wgrad<true, false>), grid, dim3(GT), 0, F->stream, Y, d.O, X, d.K, F->P, total, ppb, ktiles, F->part);
    else if (gelu_x)
        hipLaunchKernelGGL((k_wgrad<false, true>), grid, dim3(GT), 0, F->stream, Y, d.O, X, d.K, F->P, total, ppb, ktiles, F->part);
    else
        hipLaunchKernelGGL((k_wgrad<false, false>), grid, dim3(GT), 0, F->stream, Y, d.O, X, d.K, F->P, total, ppb, ktiles, F->part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(ntiles, 16), dim3(64), 0, F->stream, F->part, nblk, ntiles, ktiles, d.O,
                       d.K, F->grad + d.off);
    // bias partials in F->lpart (its loss partials were read back before the backward pass)
    hipLaunchKernelGGL(k_bgrad_part, dim3(d.O, BG_CHUNKS), dim3(GT), 0, F->stream, Y, d.O, F->P, B, F->lpart);
    hipLaunchKernelGGL(k_bgrad_reduce, dim3((d.O + 255) / 256), dim3(256), 0, F->stream, F->lpart, d.O,
                       F->grad + d.off + (int64_t)d.O * d.K);
}

// forward spectral mixing launch: MB modes per block (8 at batch 8, width 32:
// one (mode, o) per thread), LDS 2 MB B W complex <= 32 KB for every
// admissible batch and width
static void mix_fwd(pst_fno* F, int l, int B, cx<float>* vstore) {
    const int W = F->p.width;
    int MB = 2048 / (B * W);
    MB = MB < 1 ? 1 : (MB > 8 ? 8 : MB);
    const size_t sh = sizeof(cx<float>) * (2 * (size_t)MB * B * W);
    hipLaunchKernelGGL(k_mix_fwd, dim3((F->nm + MB - 1) / MB), dim3(GT), sh, F->stream, F->specA,
                       (const cx<float>*)(F->theta + F->offR[l]), F->nm, MB, B, W, W, F->specB, vstore);
}

static void forward_pass(pst_fno* F, const float* u, int B, float* out) {
    const int W = F->p.width, L = F->p.layers;
    const int64_t act = (int64_t)B * W * F->P;
    const int64_t astride = (int64_t)F->p.batch * W * F->P;  // buffers sized for the maximum batch
    float* v = F->v;
    dense_fwd(F, F->lift, false, u, B, F->theta + F->lift.off + F->lift.O * F->lift.K, nullptr, nullptr, nullptr, v,
              EPI_NONE, false);
    (void)act;
    for (int l = 0; l < L; ++l) {
        float* vl = F->v + l * astride;
        float* vn = F->v + (l + 1) * astride;
        float* sl = F->s + l * astride;
        // spectral branch: kb = c2r(R . r2c(v))
        F->fft->L->fft_r2c_modes(F->fft, vl, F->specA, B * W, F->p.modes, F->ffttmp);
        mix_fwd(F, l, B, F->vst + (int64_t)l * F->nm * F->p.batch * W);
        F->fft->L->fft_c2r_modes(F->fft, F->specB, F->kb, B * W, F->p.modes, F->ffttmp);
        const FnoDense& d = F->wc[l];
        const float* bias = F->theta + d.off + d.O * d.K;
        if (l < L - 1) dense_fwd(F, d, false, vl, B, bias, F->kb, nullptr, sl, vn, EPI_GELU, false);
        else dense_fwd(F, d, false, vl, B, bias, F->kb, nullptr, nullptr, vn, EPI_NONE, false);
    }
    float* vL = F->v + L * astride;
    dense_fwd(F, F->q1, false, vL, B, F->theta + F->q1.off + F->q1.O * F->q1.K, nullptr, nullptr, F->pre, F->pre,
              EPI_NONE, false);
    // out = u + Wq2 gelu(pre) + bq2
    dense_fwd(F, F->q2, false, F->pre, B, F->theta + F->q2.off + F->q2.O * F->q2.K, u, nullptr, nullptr, out, EPI_NONE,
              true);
}

// Inference forward on the fused layer kernels: activations ping-pong between
// the two slots of F->fact (BF16 on the matrix-core path), the x-transformed
// lines of the spectral branch stay in the transform workspace between kernels.
static void forward_fused(pst_fno* F, const float* u, int B, float* out) {
    const int W = F->p.width, L = F->p.layers, m = F->p.modes;
    void* act[2] = {F->fact, (char*)F->fact + F->fact_slot};
    fno_fused_lift(F, u, B, act[0], F->ffttmp);
    for (int l = 0; l < L; ++l) {
        F->fft->L->modes_yz_fwd(F->fft, F->specA, B * W, m, F->ffttmp);
        mix_fwd(F, l, B, nullptr);
        F->fft->L->modes_yz_inv(F->fft, F->specB, B * W, m, F->ffttmp);
        if (l < L - 1) fno_fused_layer(F, l, B, act[l & 1], act[(l + 1) & 1], F->ffttmp);
        else fno_fused_last(F, l, B, act[l & 1], F->ffttmp, u, out);
    }
}

extern "C" pst_status pst_fno_forward(pst_fno* F, const float* u, float* out, int batch) {
    if (!F) return PST_ERR_INVALID_ARG;
    if (!u || !out || batch < 1 || batch > F->p.batch) return ffail(F, PST_ERR_INVALID_ARG, "bad buffers or batch");
    if (fno_fused_supported(F->p.n)) forward_fused(F, u, batch, out);
    else forward_pass(F, u, batch, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PST_OK : ffail(F, PST_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
}

extern "C" pst_status pst_fno_loss_grad(pst_fno* F, const float* u, const float* tgt, int batch, double* loss) {
    if (!F) return PST_ERR_INVALID_ARG;
    if (!u || !tgt || batch < 1 || batch > F->p.batch) return ffail(F, PST_ERR_INVALID_ARG, "bad buffers or batch");
    const int B = batch, W = F->p.width, L = F->p.layers;
    const int64_t astride = (int64_t)F->p.batch * W * F->P, act = (int64_t)B * W * F->P;
    const int64_t per = (int64_t)3 * F->P;
    forward_pass(F, u, B, F->out);
    // loss and its gradient
    const int lb = 64;
    hipLaunchKernelGGL(k_loss_part, dim3(lb, B), dim3(GT), 0, F->stream, F->out, tgt, per, F->lpart);
    std::vector<double> part(2 * lb * B);
    if (hipMemcpyAsync(part.data(), F->lpart, sizeof(double) * part.size(), hipMemcpyDeviceToHost, F->stream) !=
            hipSuccess ||
        hipStreamSynchronize(F->stream) != hipSuccess)
        return ffail(F, PST_ERR_HIP, "loss readback failed");
    std::vector<float> coef(B);
    double Ls = 0.0;
    for (int b = 0; b < B; ++b) {
        double e2 = 0, t2 = 0;
        for (int k = 0; k < lb; ++k) {
            e2 += part[(b * lb + k) * 2];
            t2 += part[(b * lb + k) * 2 + 1];
        }
        const double en = sqrt(e2), tn = sqrt(t2);
        Ls += en / tn;
        coef[b] = (float)(en > 0 ? 1.0 / (B * en * tn) : 0.0);
    }
    if (loss) *loss = Ls / B;
    if (!isfinite(Ls)) return ffail(F, PST_ERR_NONFINITE, "loss is not finite");
    hipMemcpyAsync(F->coef, coef.data(), sizeof(float) * B, hipMemcpyHostToDevice, F->stream);
    hipLaunchKernelGGL(k_loss_grad, dim3(gs(per * B)), dim3(256), 0, F->stream, F->out, tgt, F->coef, per, B, F->dout);
    // projection: y = Wq2 gelu(pre) + bq2 + u
    dense_grad(F, F->q2, F->dout, F->pre, B, true);
    dense_fwd(F, F->q2, true, F->dout, B, nullptr, nullptr, F->pre, nullptr, F->dpre, EPI_DGELU, false);
    float* vL = F->v + L * astride;
    dense_grad(F, F->q1, F->dpre, vL, B, false);
    dense_fwd(F, F->q1, true, F->dpre, B, nullptr, nullptr, nullptr, nullptr, F->dv, EPI_NONE, false);
    const float P3 = (float)F->P;
    for (int l = L - 1; l >= 0; --l) {
        float* vl = F->v + l * astride;
        float* ds = F->ds;
        if (l < L - 1) hipLaunchKernelGGL(k_dgelu, dim3(gs(act)), dim3(256), 0, F->stream, F->dv, F->s + l * astride, ds, act);
        else ds = F->dv;
        const FnoDense& d = F->wc[l];
        dense_grad(F, d, ds, vl, B, false);
        // spectral adjoint: S = r2c(ds); g_R; tmp = c2r(conj(R)^T S)
        F->fft->L->fft_r2c_modes(F->fft, ds, F->specA, B * W, F->p.modes, F->ffttmp);
        const size_t sh = sizeof(cx<float>) * (2 * (size_t)B * W + (size_t)W * W);
        hipLaunchKernelGGL(k_mix_bwd, dim3(F->nm), dim3(GT), sh, F->stream, F->specA,
                           (const cx<float>*)(F->theta + F->offR[l]), F->vst + (int64_t)l * F->nm * F->p.batch * W,
                           F->modeoff, F->modew, F->fsz, B, W, W, P3, F->specB, (cx<float>*)(F->grad + F->offR[l]));
        F->fft->L->fft_c2r_modes(F->fft, F->specB, F->tmp, B * W, F->p.modes, F->ffttmp);
        // dv_l = Wc^T ds + tmp  (F->dv may alias ds for the last layer: write to a separate buffer)
        float* dst = (ds == F->dv) ? F->ds : F->dv;
        dense_fwd(F, d, true, ds, B, nullptr, F->tmp, nullptr, nullptr, dst, EPI_NONE, false);
        if (dst != F->dv)
            hipMemcpyAsync(F->dv, dst, 4 * act, hipMemcpyDeviceToDevice, F->stream);
    }
    dense_grad(F, F->lift, F->dv, u, B, false);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PST_OK : ffail(F, PST_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
}

extern "C" pst_status pst_fno_adam(pst_fno* F, float lr, float beta1, float beta2, float eps) {
    if (!F) return PST_ERR_INVALID_ARG;
    F->adam_t++;
    const float bc1 = 1.f - powf(beta1, (float)F->adam_t), bc2 = 1.f - powf(beta2, (float)F->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(gs(F->nparam)), dim3(256), 0, F->stream, F->theta, F->grad, F->am, F->av,
                       F->nparam, lr, beta1, beta2, eps, bc1, bc2);
    pack_all(F);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PST_OK : ffail(F, PST_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
}

extern "C" pst_status pst_fno_train_step(pst_fno* F, const float* u, const float* tgt, int batch, float lr,
                                         double* loss) {
    pst_status s = pst_fno_loss_grad(F, u, tgt, batch, loss);
    if (s) return s;
    return pst_fno_adam(F, lr, 0.9f, 0.999f, 1e-8f);
}
