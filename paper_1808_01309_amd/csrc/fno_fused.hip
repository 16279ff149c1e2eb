// Fused inference kernels of the Fourier neural operator.
//
// A layer is  s = Wc v + b + K(v),  K(v) = c2r(R . r2c(v) on the retained
// modes).  The y and z passes of the pruned transforms and the per-mode mixing
// need whole planes and run as separate kernels; everything that is local to
// one x line runs in one kernel per layer, over blocks of RB consecutive
// (b, z, y) rows and all channels:
//
//   x c2r of the spectral branch (t1 -> LDS)  ->  channel mixing Wc v on the
//   matrix cores (BF16 operands, FP32 accumulation; FP32 FMA variant)  ->
//   + bias + spectral branch, GELU  ->  store v_{l+1}  ->  x r2c of v_{l+1}
//   keeping kx < m (LDS -> t1, in place: a block reads and writes only its
//   own rows).
//
// The first kernel applies the lift instead of a layer; the last fuses the
// projection 32 -> hidden -> GELU -> 3 and the residual, so v_L and the hidden
// activations never reach HBM.  Between layers the activations are stored
// point-major, [b][point][channel] with the channels padded to a multiple of
// 16 (zeros), in BF16 on the matrix-core path (exactly the values its MFMA
// operands take: each lane's eight consecutive channels are one 16-byte
// load) and FP32 otherwise; they are written from LDS after the epilogue,
// eight channels of a point per lane, so that a wavefront stores whole points
// contiguously.  The spectral branch always transforms the FP32 values.  The matrix-core
// path uses gfx950's v_mfma_f32_32x32x16_bf16 (K = 16 per instruction), and
// its activation operands are loaded before the spectral branch's transform,
// so that their latency overlaps it.
#include "fno_internal.h"
#include "kernels.h"

namespace pst {
namespace {

constexpr int FT = 256;  // threads per block

// rows per block: RB n points, a multiple of 32 (one MFMA tile), n % RB == 0
template <int N> constexpr int fno_rows() { return N <= 16 ? 8 : (N <= 32 ? 4 : (N <= 64 ? 2 : 1)); }

template <bool BF> struct Act;
template <> struct Act<true> {
    using T = __bf16;
};
template <> struct Act<false> {
    using T = float;
};

// X, the block's values in LDS: channel c's RB rows at X[c PXS + r n + x].  The
// row stride PXS = RB n + 1 puts the channels of one point on distinct banks
// (the activation store phase reads 8 channels of a point per lane).
template <int N> constexpr int xstride() { return fno_rows<N>() * N + 1; }
// floats of X, rounded up so that the FFT line scratch after it is 16-byte aligned
template <int N> __host__ __device__ constexpr int xfloats(int W) { return (W * xstride<N>() + 3) / 4 * 4; }
// bytes of dynamic LDS: X, then one FFT line scratch per pair slot
template <int N> size_t fused_lds(int W) {
    return sizeof(float) * (size_t)xfloats<N>(W) + sizeof(cx<float>) * (size_t)(FT / NCfg<N>::G) * LineLds<float>::size(N);
}

// Block geometry: blockIdx.x = (b N + z) (N / RB) + yb, first point p0 of the
// block in a field; the block's lines (row r, channel c) live at X[c PXS + r N + x].
struct RowBlock {
    int b, z, y0;
    int64_t p0;
};
template <int N> __device__ __forceinline__ RowBlock row_block() {
    constexpr int RB = fno_rows<N>();
    RowBlock r;
    const int yb = blockIdx.x % (N / RB), bz = blockIdx.x / (N / RB);
    r.z = bz % N;
    r.b = bz / N;
    r.y0 = yb * RB;
    r.p0 = ((int64_t)r.z * N + r.y0) * N;
    return r;
}
// Line l of a block is row r = l % RB of channel c = l / RB: the two lines of a
// pair are adjacent rows of one channel (RB even), whose t1 segments are contiguous.
template <int N> __device__ __forceinline__ int64_t t1_line(const RowBlock& rb, int W, int m, int l) {
    constexpr int RB = fno_rows<N>();
    const int r = l % RB, c = l / RB;
    return ((((int64_t)rb.b * W + c) * N + rb.z) * N + rb.y0 + r) * m;
}
template <int N> __device__ __forceinline__ int x_line(int l) {
    constexpr int RB = fno_rows<N>();
    return (l / RB) * xstride<N>() + (l % RB) * N;  // X[c PXS + r N + x]
}

// x r2c of the block's RB W lines held in X, keeping kx < m, into t1.
// Lines are transformed in pairs (2i, 2i + 1) packed as one complex line.
template <int N>
__device__ __forceinline__ void rows_r2c(const float* X, int W, int m, const RowBlock& rb, cx<float>* __restrict__ t1,
                                         const cx<float>* __restrict__ tw, cx<float>* fl) {
    using C = NCfg<N>;
    using F = Fft<float, typename C::P, C::G, false, false, false, true>;
    constexpr int G = C::G, E = F::E, NPG = FT / G, LS = LineLds<float>::size(N), PB = fno_rows<N>() * N;
    const int g = threadIdx.x % G, li = threadIdx.x / G;
    const LineLds<float> lds{fl + li * LS};
    const int NL = fno_rows<N>() * W, npair = (NL + 1) / 2;
    for (int base = 0; base < npair; base += NPG) {  // same trip count in every thread
        const int l0 = 2 * (base + li), l1 = l0 + 1;
        const bool a0 = l0 < NL, a1 = l1 < NL;
        const float* x0 = X + (a0 ? x_line<N>(l0) : 0);
        const float* x1 = X + (a1 ? x_line<N>(l1) : 0);
        cx<float> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = F::first_pos(g, e);
            v[e] = {a0 ? x0[p] : 0.f, a1 ? x1[p] : 0.f};
        }
        F::run(v, g, lds, tw);
#pragma unroll
        for (int e = 0; e < E; ++e) lds(F::last_pos(g, e)) = v[e];
        __syncthreads();
        cx<float>* o0 = t1 + (a0 ? t1_line<N>(rb, W, m, l0) : 0);
        cx<float>* o1 = t1 + (a1 ? t1_line<N>(rb, W, m, l1) : 0);
        for (int k = g; k < m; k += G) {
            const cx<float> z1 = lds(k), z2 = lds(k == 0 ? 0 : N - k);
            if (a0) o0[k] = {0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y)};
            if (a1) o1[k] = {0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x)};
        }
        __syncthreads();  // the scratch is rewritten by the next pair
    }
}

// x c2r of the block's lines from t1 (kx < m, Hermitian extension, imaginary
// part of kx = 0 dropped) into X.
template <int N>
__device__ __forceinline__ void rows_c2r(const cx<float>* __restrict__ t1, int W, int m, const RowBlock& rb, float* X,
                                         const cx<float>* __restrict__ tw, cx<float>* fl) {
    using C = NCfg<N>;
    using F = Fft<float, typename C::P, C::G, true, false, false, true>;
    constexpr int G = C::G, E = F::E, NPG = FT / G, LS = LineLds<float>::size(N), PB = fno_rows<N>() * N;
    const int g = threadIdx.x % G, li = threadIdx.x / G;
    const LineLds<float> lds{fl + li * LS};
    const int NL = fno_rows<N>() * W, npair = (NL + 1) / 2;
    for (int base = 0; base < npair; base += NPG) {
        const int l0 = 2 * (base + li), l1 = l0 + 1;
        const bool a0 = l0 < NL, a1 = l1 < NL;
        const cx<float>* i0 = t1 + (a0 ? t1_line<N>(rb, W, m, l0) : 0);
        const cx<float>* i1 = t1 + (a1 ? t1_line<N>(rb, W, m, l1) : 0);
        cx<float> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = F::first_pos(g, e);
            const int k = p < m ? p : (p > N - m ? N - p : -1);
            cx<float> A = czero<float>(), B = czero<float>();
            if (k >= 0) {
                if (a0) A = i0[k];
                if (a1) B = i1[k];
            }
            if (p == 0) v[e] = {A.x, B.x};
            else if (p < m) v[e] = {A.x - B.y, A.y + B.x};
            else v[e] = {A.x + B.y, B.x - A.y};  // zero when k < 0
        }
        F::run(v, g, lds, tw);
        float* x0 = X + (a0 ? x_line<N>(l0) : 0);
        float* x1 = X + (a1 ? x_line<N>(l1) : 0);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = F::last_pos(g, e);
            if (a0) x0[q] = v[e].x;
            if (a1) x1[q] = v[e].y;
        }
        // the transform's last LDS reads precede its final barrier: the
        // scratch can be rewritten by the next pair without another one
    }
}

// Channel mixing of one tile: acc[r] = sum_k W[ot 32 + m(r)][k] x[k][n] over
// k < K for this lane's point n, in the MFMA 32x32 register layout
// m(r) = 8 (r / 4) + 4 kg + r % 4 (kg = lane / 32).  The 32x32x16 BF16 operands:
// lane n + 32 kg holds A[m = n][k] and B[k][n] for k = 16 s + 8 kg + j,
// j < 8, in K steps s (K <= 64: at most 4 steps).
constexpr int KS_MAX = 4;
struct BOps {
    bf16x8v b[KS_MAX];
};
// from stored BF16 activations of one point (channel-contiguous): one 16-byte load per step
template <int KS>
__device__ __forceinline__ void load_bops_act(BOps& o, const __bf16* __restrict__ x, int ks, int kg) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        if (s >= ks) break;
        o.b[s] = *(const bf16x8v*)(x + 16 * s + 8 * kg);
    }
}
// from FP32 values with channel stride xs (LDS); channels >= K read as zero
template <int KS>
__device__ __forceinline__ void load_bops_f32(BOps& o, const float* x, int64_t xs, int K, int ks, int kg) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        if (s >= ks) break;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 16 * s + 8 * kg + j;
            o.b[s][j] = (__bf16)(k < K ? x[k * xs] : 0.f);
        }
    }
}
template <int KS>
__device__ __forceinline__ f32x16 mfma_tile(const BOps& o, const __bf16* __restrict__ Wb, int Kpad, int ks, int ot,
                                            int n, int kg) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const __bf16* wrow = Wb + (int64_t)(ot * 32 + n) * Kpad + 8 * kg;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        if (s >= ks) break;
        const bf16x8v a = *(const bf16x8v*)(wrow + 16 * s);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, o.b[s], acc, 0, 0, 0);
    }
    return acc;
}
// FP32 FMA variant, same register layout (W FP32 [.][Kpad]; x[k xs] for k < K)
__device__ __forceinline__ f32x16 fma_tile(const float* __restrict__ Wf, int Kpad, int K, int ot, const float* x,
                                           int64_t xs, int kg) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int k = 0; k < K; ++k) {
        const float xv = x[k * xs];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] += Wf[(int64_t)(ot * 32 + 8 * (r / 4) + 4 * kg + (r % 4)) * Kpad + k] * xv;
    }
    return acc;
}

// Store the block's activations from X (FP32, after a barrier) to HBM,
// point-major: a lane writes 8 consecutive channels of one point (16 bytes,
// zeros past W), so that a wavefront's store covers whole points contiguously.
template <int N, bool BF>
__device__ __forceinline__ void store_act(const float* X, int W, typename Act<BF>::T* __restrict__ vb) {
    constexpr int PB = fno_rows<N>() * N, PXS = xstride<N>();
    if constexpr (BF) {
        const int G8 = fno_act_cp(W, true) / 8;
        for (int i = threadIdx.x; i < G8 * PB; i += FT) {
            const int pt = i / G8, og = i % G8;
            bf16x8v q;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c = 8 * og + j;
                q[j] = (__bf16)(c < W ? X[c * PXS + pt] : 0.f);
            }
            *(bf16x8v*)(vb + ((int64_t)pt * G8 + og) * 8) = q;
        }
    } else {
        for (int i = threadIdx.x; i < W * PB; i += FT) {
            const int pt = i / W, c = i % W;
            vb[(int64_t)pt * W + c] = X[c * PXS + pt];
        }
    }
}

template <int N, bool BF>
__global__ __launch_bounds__(FT) void k_fno_lift(const float* __restrict__ u, const float* __restrict__ Wl,
                                                 const float* __restrict__ bl, int W, int m,
                                                 typename Act<BF>::T* __restrict__ vout, cx<float>* __restrict__ t1,
                                                 const cx<float>* __restrict__ tw) {
    constexpr int PB = fno_rows<N>() * N, PXS = xstride<N>();
    constexpr int64_t P3 = (int64_t)N * N * N;
    extern __shared__ float X[];
    cx<float>* fl = (cx<float>*)(X + xfloats<N>(W));
    const RowBlock rb = row_block<N>();
    const float* ub = u + (int64_t)rb.b * 3 * P3 + rb.p0;
    const int CP = fno_act_cp(W, BF);
    typename Act<BF>::T* vb = vout + ((int64_t)rb.b * P3 + rb.p0) * CP;
    // consecutive threads take consecutive points (distinct LDS banks)
    for (int i = threadIdx.x; i < W * PB; i += FT) {
        const int o = i / PB, pt = i % PB;
        X[o * PXS + pt] = bl[o] + Wl[3 * o] * ub[pt] + Wl[3 * o + 1] * ub[P3 + pt] + Wl[3 * o + 2] * ub[2 * P3 + pt];
    }
    __syncthreads();
    store_act<N, BF>(X, W, vb);
    rows_r2c<N>(X, W, m, rb, t1, tw, fl);
}

struct ProjArgs {
    const __bf16* Wb;  // Wq1 padded [Hpad][Kpad] BF16
    const float* Wf;   // same, FP32
    int Kpad, H, Hpad;
    const float *bq1, *Wq2, *bq2;  // Wq2 [3][H]
    const float* u;
    float* out;
};

// KS: MFMA K steps compiled for (2: K <= 32, 4: K <= 64); ks = Kpad / 16 at run time.
template <int N, bool BF, bool LAST, int KS>
__global__ __launch_bounds__(FT) void k_fno_layer(const typename Act<BF>::T* __restrict__ vin,
                                                  const __bf16* __restrict__ Wb, const float* __restrict__ Wf,
                                                  int Kpad, int Opad, const float* __restrict__ bias, int W, int m,
                                                  typename Act<BF>::T* __restrict__ vout, cx<float>* __restrict__ t1,
                                                  const cx<float>* __restrict__ tw, ProjArgs pa) {
    constexpr int PB = fno_rows<N>() * N, PT = PB / 32, PXS = xstride<N>();
    constexpr int64_t P3 = (int64_t)N * N * N;
    static_assert(PT <= FT / 64, "one 32-point tile per wavefront");
    static_assert(sizeof(float) * 4 * 256 <= sizeof(cx<float>) * (FT / NCfg<N>::G) * LineLds<float>::size(N),
                  "projection weights (hidden <= 256) must fit in the FFT scratch");
    extern __shared__ float X[];
    cx<float>* fl = (cx<float>*)(X + xfloats<N>(W));
    const RowBlock rb = row_block<N>();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = lane & 31, kg = lane >> 5;
    const int CP = fno_act_cp(W, BF), ks = Kpad / 16;
    // this wavefront's tile: points pt0 .. pt0 + 31 of the block, every output channel
    const bool tile = wave < PT;
    const int pt0 = wave * 32;
    const int64_t gp = (int64_t)rb.b * P3 + rb.p0 + pt0 + n;   // this lane's point
    const typename Act<BF>::T* vp = vin + gp * CP;

    // the mixing's activation operands, in flight while the spectral branch is transformed
    BOps ops;
    if constexpr (BF) {
        if (tile) load_bops_act<KS>(ops, vp, ks, kg);
    }

    // spectral branch of every line of the block
    rows_c2r<N>(t1, W, m, rb, X, tw, fl);
    __syncthreads();
    float* wl = (float*)fl;  // last layer: [bq1; Wq2] (4 H floats) in the now unused FFT scratch
    if constexpr (LAST) {
        for (int i = threadIdx.x; i < 4 * pa.H; i += FT)
            wl[i] = i < pa.H ? pa.bq1[i] : pa.Wq2[i - pa.H];
    }

    // channel mixing + bias + spectral branch (+ GELU), tiles of 32 channels x 32 points
    if (tile) {
        for (int ot = 0; ot < Opad / 32; ++ot) {
            f32x16 acc;
            if constexpr (BF) acc = mfma_tile<KS>(ops, Wb, Kpad, ks, ot, n, kg);
            else acc = fma_tile(Wf, Kpad, W, ot, vp, 1, kg);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o0 = ot * 32 + 8 * i + 4 * kg;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int o = o0 + j;
                    if (o < W) {
                        float* xo = X + o * PXS + pt0 + n;
                        float s = acc[4 * i + j] + bias[o] + *xo;
                        if (!LAST) s = gelu_f(s);
                        *xo = s;  // this lane is the only reader and writer of X[o][pt]
                    }
                }
            }
        }
    }
    __syncthreads();

    if constexpr (!LAST) {
        store_act<N, BF>(X, W, vout + ((int64_t)rb.b * P3 + rb.p0) * CP);
        rows_r2c<N>(X, W, m, rb, t1, tw, fl);
    } else if (tile) {
        // projection out = u + Wq2 gelu(Wq1 v + bq1) + bq2 on this wave's tile;
        // bq1 and Wq2 were staged in LDS (the FFT scratch)
        BOps pops;
        if constexpr (BF) load_bops_f32<KS>(pops, X + pt0 + n, (int64_t)PXS, W, pa.Kpad / 16, kg);
        float y0 = 0.f, y1 = 0.f, y2 = 0.f;
        for (int ht = 0; ht < pa.Hpad / 32; ++ht) {
            f32x16 acc;
            if constexpr (BF) acc = mfma_tile<KS>(pops, pa.Wb, pa.Kpad, pa.Kpad / 16, ht, n, kg);
            else acc = fma_tile(pa.Wf, pa.Kpad, W, ht, X + pt0 + n, (int64_t)PXS, kg);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // hidden units h0 .. h0 + 3 (consecutive): their bias and output
                // weights as one 16-byte LDS read each where aligned
                const int h0 = ht * 32 + 8 * i + 4 * kg;
                if (h0 + 4 <= pa.H && pa.H % 4 == 0) {
                    const float4 bq = *(const float4*)(wl + h0);
                    const float4 w0 = *(const float4*)(wl + pa.H + h0);
                    const float4 w1 = *(const float4*)(wl + 2 * pa.H + h0);
                    const float4 w2 = *(const float4*)(wl + 3 * pa.H + h0);
                    const float a0 = gelu_f(acc[4 * i] + bq.x), a1 = gelu_f(acc[4 * i + 1] + bq.y);
                    const float a2 = gelu_f(acc[4 * i + 2] + bq.z), a3 = gelu_f(acc[4 * i + 3] + bq.w);
                    y0 += w0.x * a0 + w0.y * a1 + w0.z * a2 + w0.w * a3;
                    y1 += w1.x * a0 + w1.y * a1 + w1.z * a2 + w1.w * a3;
                    y2 += w2.x * a0 + w2.y * a1 + w2.z * a2 + w2.w * a3;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int h = h0 + j;
                        if (h >= pa.H) continue;
                        const float a = gelu_f(acc[4 * i + j] + wl[h]);
                        y0 += wl[pa.H + h] * a;
                        y1 += wl[2 * pa.H + h] * a;
                        y2 += wl[3 * pa.H + h] * a;
                    }
                }
            }
        }
        // the two half-waves hold disjoint hidden units of the same points
        y0 += __shfl_xor(y0, 32);
        y1 += __shfl_xor(y1, 32);
        y2 += __shfl_xor(y2, 32);
        if (kg == 0) {
            const int64_t i0 = (int64_t)rb.b * 3 * P3 + rb.p0 + pt0 + n;
            pa.out[i0] = pa.u[i0] + y0 + pa.bq2[0];
            pa.out[i0 + P3] = pa.u[i0 + P3] + y1 + pa.bq2[1];
            pa.out[i0 + 2 * P3] = pa.u[i0 + 2 * P3] + y2 + pa.bq2[2];
        }
    }
}

template <int N>
struct Fused {
    static unsigned grid(int B) { return (unsigned)(B * N * (N / fno_rows<N>())); }
    static void lift(pst_fno* F, const float* u, int B, void* act, cx<float>* t1) {
        const int W = F->p.width;
        const float* Wl = F->theta + F->lift.off;
        const cx<float>* tw = (const cx<float>*)F->fft->tw;
        if (F->p.mfma)
            hipLaunchKernelGGL((k_fno_lift<N, true>), dim3(grid(B)), dim3(FT), fused_lds<N>(W), F->stream, u, Wl,
                               Wl + 3 * W, W, F->p.modes, (__bf16*)act, t1, tw);
        else
            hipLaunchKernelGGL((k_fno_lift<N, false>), dim3(grid(B)), dim3(FT), fused_lds<N>(W), F->stream, u, Wl,
                               Wl + 3 * W, W, F->p.modes, (float*)act, t1, tw);
    }
    template <bool LAST, int KS>
    static void layer_ks(pst_fno* F, const FnoDense& d, const float* bias, int B, const void* ain, void* aout,
                         cx<float>* t1, const cx<float>* tw, const ProjArgs& pa) {
        const int W = F->p.width;
        if (F->p.mfma)
            hipLaunchKernelGGL((k_fno_layer<N, true, LAST, KS>), dim3(grid(B)), dim3(FT), fused_lds<N>(W), F->stream,
                               (const __bf16*)ain, (const __bf16*)d.Wb, d.Wf, d.Kpad, d.Opad, bias, W, F->p.modes,
                               (__bf16*)aout, t1, tw, pa);
        else
            hipLaunchKernelGGL((k_fno_layer<N, false, LAST, KS>), dim3(grid(B)), dim3(FT), fused_lds<N>(W),
                               F->stream, (const float*)ain, (const __bf16*)d.Wb, d.Wf, d.Kpad, d.Opad, bias, W,
                               F->p.modes, (float*)aout, t1, tw, pa);
    }
    template <bool LAST>
    static void layer(pst_fno* F, int l, int B, const void* ain, void* aout, cx<float>* t1, const float* u, float* out) {
        const FnoDense& d = F->wc[l];
        const float* bias = F->theta + d.off + (int64_t)d.O * d.K;
        const cx<float>* tw = (const cx<float>*)F->fft->tw;
        ProjArgs pa{};
        if (LAST) {
            const FnoDense& q1 = F->q1;
            const FnoDense& q2 = F->q2;
            pa.Wb = (const __bf16*)q1.Wb;
            pa.Wf = q1.Wf;
            pa.Kpad = q1.Kpad;
            pa.H = q1.O;
            pa.Hpad = q1.Opad;
            pa.bq1 = F->theta + q1.off + (int64_t)q1.O * q1.K;
            pa.Wq2 = F->theta + q2.off;
            pa.bq2 = F->theta + q2.off + (int64_t)q2.O * q2.K;
            pa.u = u;
            pa.out = out;
        }
        // the layer's and the projection's K (both the width) in steps of 16
        if (d.Kpad <= 32) layer_ks<LAST, 2>(F, d, bias, B, ain, aout, t1, tw, pa);
        else layer_ks<LAST, 4>(F, d, bias, B, ain, aout, t1, tw, pa);
    }
};

}  // namespace

#define FNO_FUSED_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

bool fno_fused_supported(int n) {
#define FNO_CASE(N) if (n == N) return true;
    FNO_FUSED_SIZES(FNO_CASE)
#undef FNO_CASE
    return false;
}

void fno_fused_lift(pst_fno* F, const float* u, int B, void* act, cx<float>* t1) {
#define FNO_CASE(N) if (F->p.n == N) return Fused<N>::lift(F, u, B, act, t1);
    FNO_FUSED_SIZES(FNO_CASE)
#undef FNO_CASE
}

void fno_fused_layer(pst_fno* F, int l, int B, const void* act_in, void* act_out, cx<float>* t1) {
#define FNO_CASE(N) if (F->p.n == N) return Fused<N>::template layer<false>(F, l, B, act_in, act_out, t1, nullptr, nullptr);
    FNO_FUSED_SIZES(FNO_CASE)
#undef FNO_CASE
}

void fno_fused_last(pst_fno* F, int l, int B, const void* act_in, cx<float>* t1, const float* u, float* out) {
#define FNO_CASE(N) if (F->p.n == N) return Fused<N>::template layer<true>(F, l, B, act_in, nullptr, t1, u, out);
    FNO_FUSED_SIZES(FNO_CASE)
#undef FNO_CASE
}

}  // namespace pst
