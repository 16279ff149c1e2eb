// Host runtime of the C ABI (include/pst.h): plan life cycle, state I/O,
// time stepping, diagnostics, standalone transforms and timers, plus the
// size-independent kernels (gather / scatter between the ABI spectral layout
// and the dealiased compact state, FP64 reductions).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <algorithm>
#include <string>

#include "fft_engine.h"
#include "plan.h"

using namespace pst;

// --------------------------------------------------------------- registry
namespace pst {
#define PST_DECL_N(NV) const Launchers* launchers_n##NV(int precision);
PST_DECL_N(16) PST_DECL_N(24) PST_DECL_N(32) PST_DECL_N(48) PST_DECL_N(64) PST_DECL_N(96)
PST_DECL_N(128) PST_DECL_N(256) PST_DECL_N(512) PST_DECL_N(1024)
#undef PST_DECL_N

const Launchers* launchers_for(int n, int precision) {
    switch (n) {
        case 16: return launchers_n16(precision);
        case 24: return launchers_n24(precision);
        case 32: return launchers_n32(precision);
        case 48: return launchers_n48(precision);
        case 64: return launchers_n64(precision);
        case 96: return launchers_n96(precision);
        case 128: return launchers_n128(precision);
        case 256: return launchers_n256(precision);
        case 512: return launchers_n512(precision);
        case 1024: return launchers_n1024(precision);
        default: return nullptr;
    }
}
}  // namespace pst

// --------------------------------------------------------------- errors
static thread_local std::string g_create_err;

static pst_status fail(pst_plan* P, pst_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (P) P->err = buf;
    else g_create_err = buf;
    return s;
}

#define HIPCHK(P, call)                                                                           \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail((P), PST_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

static pst_status check_launch(pst_plan* P, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(P, PST_ERR_HIP, "%s: kernel launch failed: %s", what, hipGetErrorString(e));
    return PST_OK;
}

extern "C" const char* pst_status_str(pst_status s) {
    switch (s) {
        case PST_OK: return "ok";
        case PST_ERR_INVALID_ARG: return "invalid argument";
        case PST_ERR_UNSUPPORTED_N: return "unsupported grid size";
        case PST_ERR_OOM: return "out of device memory";
        case PST_ERR_HIP: return "HIP runtime error";
        case PST_ERR_NONFINITE: return "non-finite value";
        case PST_ERR_UNSUPPORTED: return "unsupported option";
    }
    return "unknown status";
}

extern "C" const char* pst_last_error(const pst_plan* P) { return P ? P->err.c_str() : g_create_err.c_str(); }

extern "C" int pst_supported_n(int n) {
    switch (n) {
        case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 256: case 512: case 1024: return 1;
        default: return 0;
    }
}

static void fft3_c2r(pst_plan* P, const void* in, void* out, int nf, void* tmp);

// --------------------------------------------------------------- c2r without allocation
// Device memory of pst_fft_c2r_noalloc: the n roots of unity followed by the
// workspace of the z and y passes.  One copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in: kernels are given
// the per-device address from hipGetSymbolAddress, never the symbol itself.
static __device__ __align__(256) unsigned char scratch[PST_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEV];

// Address of this device's copy of `scratch` (looked up once per device,
// with that device current).
pst_status scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEV)
        return fail(nullptr, PST_ERR_HIP, "no current HIP device (or device index %d too large)", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(nullptr, PST_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PST_OK;
}
}  // namespace

// tw[m] = exp(-2 pi i m / n), evaluated in FP64 and rounded once to T
template <typename T>
__global__ void k_roots(cx<T>* __restrict__ tw, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double sn, cs;
    sincospi(2.0 * (double)m / (double)n, &sn, &cs);
    tw[m] = {(T)cs, (T)(-sn)};
}

extern "C" size_t pst_fft_c2r_noalloc_bytes(int n, int precision, int nfields) {
    if (!pst_supported_n(n) || (precision != PST_FP32 && precision != PST_FP64) || nfields < 1) return 0;
    const size_t es = precision == PST_FP64 ? 16 : 8, un = (size_t)n;
    const size_t tw = (un * es + 255) / 256 * 256;
    return tw + (size_t)nfields * un * un * (un / 2 + 1) * es;
}

extern "C" pst_status pst_fft_c2r_noalloc(int n, int precision, const void* in, void* out, int nfields,
                                          void* hip_stream) {
    if (!in || !out) return fail(nullptr, PST_ERR_INVALID_ARG, "NULL buffer");
    if (precision != PST_FP32 && precision != PST_FP64)
        return fail(nullptr, PST_ERR_INVALID_ARG, "precision %d", precision);
    if (nfields < 1) return fail(nullptr, PST_ERR_INVALID_ARG, "nfields < 1");
    if (!pst_supported_n(n)) return fail(nullptr, PST_ERR_UNSUPPORTED_N, "n = %d not supported", n);
    const size_t need = pst_fft_c2r_noalloc_bytes(n, precision, nfields);
    if (need > (size_t)PST_NOALLOC_SCRATCH_BYTES)
        return fail(nullptr, PST_ERR_INVALID_ARG,
                    "n = %d with %d field(s) needs %zu bytes of scratch; the limit is %zu", n, nfields, need,
                    (size_t)PST_NOALLOC_SCRATCH_BYTES);
    const Launchers* L = launchers_for(n, precision);
    if (!L) return fail(nullptr, PST_ERR_UNSUPPORTED_N, "n = %d has no kernels", n);
    void* base = nullptr;
    pst_status s = scratch_address(&base);
    if (s) return s;
    const size_t es = precision == PST_FP64 ? 16 : 8;
    void* tmp = (unsigned char*)base + (need - (size_t)nfields * n * n * (n / 2 + 1) * es);
    // a plan shell on the stack: the launchers read only the stream, the
    // twiddle pointer and the (cleared) timer flag from it
    pst_plan Q{};
    Q.p.n = n;
    Q.p.precision = precision;
    Q.p.flags = 0;
    Q.stream = (hipStream_t)hip_stream;
    Q.geo = make_geo(n, n, n, 0, 0, 0, 1.0, 1.0, 1.0, 0);
    Q.L = Q.Lx = Q.Ly = L;
    Q.tw = Q.twx = Q.twy = base;
    Q.esz = es;
    if (precision == PST_FP64)
        hipLaunchKernelGGL(k_roots<double>, dim3((n + 255) / 256), dim3(256), 0, Q.stream, (cx<double>*)base, n);
    else
        hipLaunchKernelGGL(k_roots<float>, dim3((n + 255) / 256), dim3(256), 0, Q.stream, (cx<float>*)base, n);
    // every element of the workspace is written by the z pass before it is read
    fft3_c2r(&Q, in, out, nfields, tmp);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, PST_ERR_HIP, "fft_c2r_noalloc: kernel launch failed: %s", hipGetErrorString(e));
    return PST_OK;
}

// --------------------------------------------------------------- timers
namespace pst {
KTimer::KTimer(pst_plan* plan, int k) : P(plan), kind(k) {
    if (!(P->p.flags & PST_FLAG_TIMERS)) return;
    for (hipEvent_t* ev : {&a, &b}) {
        if (!P->pool.empty()) {
            *ev = P->pool.back();
            P->pool.pop_back();
        } else if (hipEventCreate(ev) != hipSuccess) {
            *ev = nullptr;
        }
    }
    if (a) hipEventRecord(a, P->stream);
}
KTimer::~KTimer() {
    if (!(P->p.flags & PST_FLAG_TIMERS) || !a || !b) return;
    hipEventRecord(b, P->stream);
    P->pending.push_back({kind, a, b});
}
}  // namespace pst

static void drain_timers(pst_plan* P) {
    for (auto& r : P->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            P->t_ms[r.kind] += ms;
            P->t_cnt[r.kind] += 1;
        }
        P->pool.push_back(r.a);
        P->pool.push_back(r.b);
    }
    P->pending.clear();
}

// --------------------------------------------------------------- small kernels
// ABI spectral layout [c][nz][ny][nxh] (nxh = nx/2 + 1, or nx for a complex
// field) <-> compact kept modes [c][jx][jy][jz].
template <typename T>
__global__ void k_gather(const cx<T>* __restrict__ abi, cx<T>* __restrict__ st, Geo g, int ncomp) {
    const int64_t total = (int64_t)ncomp * g.sc;
    const int nx = g.nx, ny = g.ny, nz = g.n, nxh = g.full ? nx : nx / 2 + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / g.sc);
        int64_t r = i % g.sc;
        const int jz = (int)(r % g.M);
        r /= g.M;
        const int jy = (int)(r % g.My);
        const int jx = (int)(r / g.My);
        const int ky = ky_of_j(jy, g), kz = k_of_j(jz, g);
        const int iy = (ky + ny) % ny, iz = (kz + nz) % nz;
        const cx<T>* a = abi + (int64_t)c * nz * ny * nxh;
        if (g.full) {   // whole spectrum, no symmetry: a plain copy of the kept modes
            const int ix = (kx_of_j(jx, g) + nx) % nx;
            st[i] = a[((int64_t)iz * ny + iy) * nxh + ix];
            continue;
        }
        const int kx = jx;
        cx<T> v = a[((int64_t)iz * ny + iy) * nxh + kx];
        if (kx == 0) {
            const cx<T> m = a[((int64_t)((nz - iz) % nz) * ny + (ny - iy) % ny) * nxh];
            v = {T(0.5) * (v.x + m.x), T(0.5) * (v.y - m.y)};
        }
        st[i] = v;
    }
}

template <typename T>
__global__ void k_scatter(const cx<T>* __restrict__ st, cx<T>* __restrict__ abi, Geo g, int ncomp) {
    const int nx = g.nx, ny = g.ny, nz = g.n, nxh = g.full ? nx : nx / 2 + 1;
    const int64_t per = (int64_t)nz * ny * nxh, total = (int64_t)ncomp * per;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / per);
        int64_t r = i % per;
        const int ix = (int)(r % nxh);
        r /= nxh;
        const int iy = (int)(r % ny), iz = (int)(r / ny);
        const int ky = k_of_pos(iy, ny), kz = k_of_pos(iz, nz);
        // full axis: signed kx, compact jx as for ky and kz
        const int kx = g.full ? k_of_pos(ix, nx) : ix;
        const int jx = g.full ? (kx >= 0 ? kx : kx + 2 * g.Kx + 1) : kx;
        cx<T> v = {T(0), T(0)};
        if (kx <= g.Kx && -kx <= g.Kx && ky <= g.Ky && -ky <= g.Ky && kz <= g.K && -kz <= g.K) {
            const int jy = ky >= 0 ? ky : ky + g.My, jz = kz >= 0 ? kz : kz + g.M;
            v = st[(int64_t)c * g.sc + ((int64_t)jx * g.My + jy) * g.M + jz];
        }
        abi[i] = v;
    }
}

// Energy partials: block b sums w |v|^2 over its grid-stride share of the
// modes of components [c0, c0 + nc) in a fixed order -> partial[b] (double).
constexpr int RED_BLOCKS = 1024, RED_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_energy_part(const cx<T>* __restrict__ st, Geo g, int c0, int nc,
                                                             double* __restrict__ part, int k2w) {
    __shared__ double sh[RED_THREADS];
    double acc = 0.0;
    const int64_t per = g.sc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (int64_t)gridDim.x * blockDim.x) {
        const int jx = (int)(i / ((int64_t)g.My * g.M));
        // half spectrum: weight 2 off the kx = 0 plane; the full spectrum counts each mode once
        const int kx = kx_of_j(jx, g);
        double w = (g.full || kx == 0) ? 1.0 : 2.0;
        if (k2w) {  // enstrophy: weight |k|^2 (physical wavenumbers)
            const int ky = ky_of_j((int)((i / g.M) % g.My), g), kz = k_of_j((int)(i % g.M), g);
            const double fx = g.ax * kx, fy = g.ay * ky, fz = g.az * kz;
            w *= fx * fx + fy * fy + fz * fz;
        }
        double s = 0.0;
        for (int c = 0; c < nc; ++c) {
            const cx<T> v = st[(int64_t)(c0 + c) * per + i];
            s += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
        acc += w * s;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(RED_THREADS) void k_sum_final(const double* __restrict__ part, int np, double* out,
                                                           double scale) {
    __shared__ double sh[RED_THREADS];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += RED_THREADS) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = scale * sh[0];
}

constexpr int MAX_SHELLS = 2048;

// shell of a mode: floor(|k| / dk + 1/2), dk the smallest a_i
__device__ __forceinline__ int shell_of(double k2, double dk) { return (int)floor(sqrt(k2) / dk + 0.5); }

// Shell spectrum with a fixed summation order (bitwise repeatable): block s
// owns shell s.  Its threads stride over the (kx, ky) lines; along a line the
// shell index grows with |kz|, so the line's modes in shell s are the |kz| of
// one contiguous range, found from an estimate and the exact test on
// floor(|k| / dk + 1/2).  Per-thread sums are then combined by a fixed tree.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_spectrum(const cx<T>* __restrict__ st, Geo g, int c0, int nc,
                                                          double* __restrict__ bins, double dk) {
    __shared__ double sh[RED_THREADS];
    const int s = blockIdx.x;
    const double hi = (s + 0.5) * dk * ((s + 0.5) * dk);
    const int64_t per = g.sc, nlines = (int64_t)g.nxk * g.My;
    double acc = 0.0;
    for (int64_t l = threadIdx.x; l < nlines; l += RED_THREADS) {
        const int jx = (int)(l / g.My), jy = (int)(l % g.My);
        const int kx = kx_of_j(jx, g), ky = ky_of_j(jy, g);
        const double fx = g.ax * kx, fy = g.ay * ky;
        const double r2 = fx * fx + fy * fy;
        if (r2 > hi) continue;   // every mode of the line lies beyond shell s
        const double lo2 = (s - 0.5) * dk * ((s - 0.5) * dk) - r2;
        int a = lo2 > 0.0 ? (int)(sqrt(lo2) / g.az) : 0;
        a = a > 0 ? a - 1 : 0;
        while (a <= g.K && shell_of(r2 + (g.az * a) * (g.az * a), dk) < s) ++a;
        // half spectrum: 1/2 w |v|^2 (energy); full spectrum: |psi|^2 (number)
        const double w = g.full ? 1.0 : 0.5 * (kx == 0 ? 1.0 : 2.0);
        const int64_t line = l * g.M;
        for (int kz = a; kz <= g.K && shell_of(r2 + (g.az * kz) * (g.az * kz), dk) == s; ++kz) {
            for (int sgn = 0; sgn < (kz == 0 ? 1 : 2); ++sgn) {
                const int jz = sgn == 0 ? kz : g.M - kz;
                double q = 0.0;
                for (int c = 0; c < nc; ++c) {
                    const cx<T> v = st[(int64_t)(c0 + c) * per + line + jz];
                    q += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
                }
                acc += w * q;
            }
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int h = RED_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) bins[s] = sh[0];
}

// --------------------------------------------------------------- helpers
static unsigned grid_for(int64_t total, int threads = 256) {
    int64_t b = (total + threads - 1) / threads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

static pst_status dalloc(pst_plan* P, void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) return PST_OK;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(P, PST_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    P->owned_bytes += bytes;
    return PST_OK;
}

static size_t abi_spec_bytes(const pst_plan* P, int ncomp) {
    const size_t nx = (size_t)P->geo.nx;
    return (size_t)ncomp * P->geo.n * P->geo.ny * (P->geo.full ? nx : nx / 2 + 1) * P->esz;
}
static size_t phys_points(const pst_plan* P) { return (size_t)P->geo.nx * P->geo.ny * P->geo.n; }

// Standalone 3D transforms composed from one pass per axis (each axis with its
// own n).  Physical [nf][nz][ny][nx], spectral [nf][nz][ny][nxh].
static void fft3_r2c(pst_plan* P, const void* in, void* out, int nf) {
    const Geo& g = P->geo;
    const int64_t nxh = g.nx / 2 + 1, plane = (int64_t)g.ny * nxh;
    P->Lx->fftx_r2c(P, in, out, (int64_t)nf * g.ny * g.n);
    P->Ly->fft_cols(P, out, out, nxh, nxh, plane, (int64_t)nf * g.n, 0, 1.0, PST_K_FFTY);
    P->L->fft_cols(P, out, out, plane, plane, plane * g.n, nf, 0, 1.0 / ((double)g.nx * g.ny * g.n), PST_K_FFTZ);
}
// c2r: in is left unchanged (the z and y passes work in tmp)
static void fft3_c2r(pst_plan* P, const void* in, void* out, int nf, void* tmp) {
    const Geo& g = P->geo;
    const int64_t nxh = g.nx / 2 + 1, plane = (int64_t)g.ny * nxh;
    P->L->fft_cols(P, in, tmp, plane, plane, plane * g.n, nf, 1, 1.0, PST_K_FFTZ);
    P->Ly->fft_cols(P, tmp, tmp, nxh, nxh, plane, (int64_t)nf * g.n, 1, 1.0, PST_K_FFTY);
    P->Lx->fftx_c2r(P, tmp, out, (int64_t)nf * g.ny * g.n);
}
// complex field: forward (sign -, 1 / (nx ny nz)) or inverse (sign +, unscaled)
static void fft3_c2c(pst_plan* P, const void* in, void* out, int nf, int inverse) {
    const Geo& g = P->geo;
    const int64_t plane = (int64_t)g.ny * g.nx;
    const double s = inverse ? 1.0 : 1.0 / ((double)g.nx * g.ny * g.n);
    P->Lx->fftx_c2c(P, in, out, (int64_t)nf * g.ny * g.n, inverse);
    P->Ly->fft_cols(P, out, out, g.nx, g.nx, plane, (int64_t)nf * g.n, inverse, 1.0, PST_K_FFTY);
    P->L->fft_cols(P, out, out, plane, plane, plane * g.n, nf, inverse, s, PST_K_FFTZ);
}

static pst_status ensure_abi(pst_plan* P, size_t bytes) {
    if (P->abi_bytes >= bytes) return PST_OK;
    if (P->abi) {
        hipStreamSynchronize(P->stream);
        hipFree(P->abi);
        P->owned_bytes -= P->abi_bytes;
        P->abi = nullptr;
        P->abi_bytes = 0;
    }
    pst_status s = dalloc(P, &P->abi, bytes);
    if (s == PST_OK) P->abi_bytes = bytes;
    return s;
}

// host tables in FP64, rounded once to the plan precision
template <typename T>
static pst_status upload_roots(pst_plan* P, void* dst, int n) {
    std::vector<cx<T>> tw(n);
    for (int m = 0; m < n; ++m) {
        // exp(-2 pi i m / n) evaluated in extended precision, rounded once
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
        tw[m].x = (T)cosl(a);
        tw[m].y = (T)(-sinl(a));
    }
    HIPCHK(P, hipMemcpy(dst, tw.data(), sizeof(cx<T>) * n, hipMemcpyHostToDevice));
    return PST_OK;
}

template <typename T>
static pst_status upload_tables(pst_plan* P) {
    const int n = P->p.n;
    // integer |k|^2 indexes the integrating factors on the 2 pi box; other
    // boxes evaluate them per mode (the tables stay unused there)
    const int K = std::max(P->geo.K, std::max(P->geo.Kx, P->geo.Ky));
    pst_status s = upload_roots<T>(P, P->tw, n);
    if (!s && P->twy != P->tw) s = upload_roots<T>(P, P->twy, P->geo.ny);
    if (!s && P->twx != P->tw && P->twx != P->twy) s = upload_roots<T>(P, P->twx, P->geo.nx);
    if (s) return s;
    const int nk2 = 3 * K * K + 1;
    if (P->p.solver == PST_GPE) {
        // exp(-i alpha |k|^2 h / 2) and its square, by integer |k|^2
        std::vector<cx<T>> E(nk2), E2(nk2);
        for (int k2 = 0; k2 < nk2; ++k2) {
            const double a = P->p.alpha * (double)k2 * P->p.dt;
            E[k2] = {(T)cos(0.5 * a), (T)(-sin(0.5 * a))};
            E2[k2] = {(T)cos(a), (T)(-sin(a))};
        }
        HIPCHK(P, hipMemcpy(P->Etab[0], E.data(), sizeof(cx<T>) * nk2, hipMemcpyHostToDevice));
        HIPCHK(P, hipMemcpy(P->E2tab[0], E2.data(), sizeof(cx<T>) * nk2, hipMemcpyHostToDevice));
        return PST_OK;
    }
    for (int grp = 0; grp < 2; ++grp) {
        const double visc = grp == 0 ? P->p.nu : P->p.eta;
        std::vector<T> E(nk2), E2(nk2);
        for (int k2 = 0; k2 < nk2; ++k2) {
            const double e = exp(-visc * (double)k2 * P->p.dt * 0.5);
            E[k2] = (T)e;
            E2[k2] = (T)(e * e);
        }
        HIPCHK(P, hipMemcpy(P->Etab[grp], E.data(), sizeof(T) * nk2, hipMemcpyHostToDevice));
        HIPCHK(P, hipMemcpy(P->E2tab[grp], E2.data(), sizeof(T) * nk2, hipMemcpyHostToDevice));
    }
    return PST_OK;
}

// --------------------------------------------------------------- plan
static constexpr double TWO_PI = 6.28318530717958647692528676655900577;
// points and box length of axis a (0 = x, 1 = y, 2 = z); 0 selects n and 2 pi
static int ax_n(const pst_params* p, int a) {
    const int m = a == 0 ? p->nx : a == 1 ? p->ny : p->nz;
    return m > 0 ? m : p->n;
}
static double ax_len(const pst_params* p, int a) {
    const double l = a == 0 ? p->lx : a == 1 ? p->ly : p->lz;
    return l > 0.0 ? l : TWO_PI;
}

extern "C" void pst_plan_destroy(pst_plan* P) {
    if (!P) return;
    hipStreamSynchronize(P->stream);
    void* bufs[] = {P->U, P->V, P->Acc, P->A, P->B, P->C, P->tw, P->Etab[0], P->Etab[1],
                    P->E2tab[0], P->E2tab[1], P->force, P->abi, P->red};
    for (void* b : bufs)
        if (b) hipFree(b);
    if (P->twy && P->twy != P->tw) hipFree(P->twy);
    if (P->twx && P->twx != P->tw && P->twx != P->twy) hipFree(P->twx);
    for (auto& r : P->pending) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : P->pool) hipEventDestroy(e);
    delete P;
}

extern "C" pst_status pst_plan_create(const pst_params* p, void* hip_stream, pst_plan** out) {
    g_create_err.clear();
    if (!out) return fail(nullptr, PST_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(nullptr, PST_ERR_INVALID_ARG, "params is NULL");
    if (p->solver != PST_NS && p->solver != PST_MHD && p->solver != PST_BOUSSINESQ && p->solver != PST_GPE)
        return fail(nullptr, PST_ERR_INVALID_ARG, "solver %d", p->solver);
    const bool gpe = p->solver == PST_GPE;
    if (gpe && (!isfinite(p->alpha) || !isfinite(p->beta)))
        return fail(nullptr, PST_ERR_INVALID_ARG, "alpha and beta must be finite");
    if (gpe && p->dealias != PST_DEALIAS_CUBE)
        return fail(nullptr, PST_ERR_UNSUPPORTED, "the GPE solver dealiases by the cube only");
    if (p->precision != PST_FP32 && p->precision != PST_FP64)
        return fail(nullptr, PST_ERR_INVALID_ARG, "precision %d", p->precision);
    if (p->rk_order != 2 && p->rk_order != 4) return fail(nullptr, PST_ERR_INVALID_ARG, "rk_order %d", p->rk_order);
    if (!(p->dt > 0.0) || !isfinite(p->dt)) return fail(nullptr, PST_ERR_INVALID_ARG, "dt must be > 0");
    if (!gpe && (!(p->nu >= 0.0) || !isfinite(p->nu))) return fail(nullptr, PST_ERR_INVALID_ARG, "nu must be >= 0");
    if ((p->solver == PST_MHD || p->solver == PST_BOUSSINESQ) && (!(p->eta >= 0.0) || !isfinite(p->eta)))
        return fail(nullptr, PST_ERR_INVALID_ARG, "eta must be >= 0");
    if (p->solver == PST_BOUSSINESQ && !isfinite(p->nbv))
        return fail(nullptr, PST_ERR_INVALID_ARG, "nbv must be finite");
    if (p->dealias != PST_DEALIAS_CUBE && p->dealias != PST_DEALIAS_SPHERE && p->dealias != PST_DEALIAS_NONE)
        return fail(nullptr, PST_ERR_UNSUPPORTED, "dealias %d", p->dealias);
    if (p->flags & ~(unsigned)(PST_FLAG_LINEAR_ONLY | PST_FLAG_TIMERS))
        return fail(nullptr, PST_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
    for (int a = 0; a < 3; ++a) {
        const int m = a == 0 ? p->nx : a == 1 ? p->ny : p->nz;
        const double l = a == 0 ? p->lx : a == 1 ? p->ly : p->lz;
        if (m < 0) return fail(nullptr, PST_ERR_INVALID_ARG, "axis %d: %d points", a, m);
        if (!(l >= 0.0) || !isfinite(l)) return fail(nullptr, PST_ERR_INVALID_ARG, "axis %d: box length %g", a, l);
        if (m == 0 && p->n == 0) return fail(nullptr, PST_ERR_UNSUPPORTED_N, "n = 0 not supported");
        if (!pst_supported_n(ax_n(p, a)))
            return fail(nullptr, PST_ERR_UNSUPPORTED_N, "axis %d: n = %d not supported", a, ax_n(p, a));
    }
    const bool cubic = ax_n(p, 0) == ax_n(p, 2) && ax_n(p, 1) == ax_n(p, 2) && ax_len(p, 0) == TWO_PI &&
                       ax_len(p, 1) == TWO_PI && ax_len(p, 2) == TWO_PI;
    if (!cubic && p->dealias == PST_DEALIAS_SPHERE)
        return fail(nullptr, PST_ERR_UNSUPPORTED, "spherical truncation needs a cubic 2 pi grid");
    const Launchers* L = launchers_for(ax_n(p, 2), p->precision);
    const Launchers* Lx = launchers_for(ax_n(p, 0), p->precision);
    const Launchers* Ly = launchers_for(ax_n(p, 1), p->precision);
    if (!L || !Lx || !Ly) return fail(nullptr, PST_ERR_UNSUPPORTED_N, "no kernels for this grid");

    pst_plan* P = new pst_plan();
    P->p = *p;
    if (P->p.solver == PST_NS) P->p.eta = P->p.nu;
    P->stream = (hipStream_t)hip_stream;
    P->L = L;
    P->Lx = Lx;
    P->Ly = Ly;
    P->esz = p->precision == PST_FP64 ? 16 : 8;
    // per-axis cutoffs.  2/3 rule: the largest K with 3K < n; NONE keeps every
    // mode but the Nyquist; GPE (cubic product): the largest K with 4K < n, kx
    // on the full axis
    auto cut = [&](int m) {
        return gpe ? (m + 3) / 4 - 1 : p->dealias == PST_DEALIAS_NONE ? m / 2 - 1 : (m + 2) / 3 - 1;
    };
    const int nx = ax_n(p, 0), ny = ax_n(p, 1), n = ax_n(p, 2);
    P->geo = make_geo(nx, ny, n, cut(nx), cut(ny), cut(n), TWO_PI / ax_len(p, 0), TWO_PI / ax_len(p, 1),
                      TWO_PI / ax_len(p, 2), gpe ? 1 : 0);
    P->p.n = n;
    const int K = P->geo.K, M = P->geo.M;
    (void)M;
    const bool mhd = p->solver == PST_MHD, bq = p->solver == PST_BOUSSINESQ;
    // state components; fields of the backward passes (v, i k x v per vector
    // field; grad theta and theta; psi) and of the forward passes
    P->ncomp = mhd ? 6 : bq ? 4 : gpe ? 1 : 3;
    P->nfin = mhd ? 12 : bq ? 10 : gpe ? 1 : 6;
    P->nfout = mhd ? 6 : bq ? 4 : gpe ? 1 : 3;
    P->kf = -1;
    const size_t es = P->esz, tsz = p->precision == PST_FP64 ? 8 : 4;
    pst_status s = PST_OK;
#define ALLOC(ptr, bytes)                                   \
    do {                                                    \
        s = dalloc(P, (void**)&(ptr), (bytes));             \
        if (s != PST_OK) {                                  \
            g_create_err = P->err;                          \
            pst_plan_destroy(P);                            \
            return s;                                       \
        }                                                   \
    } while (0)
    const size_t st_bytes = (size_t)P->ncomp * P->geo.sc * es;
    ALLOC(P->U, st_bytes);
    ALLOC(P->V, st_bytes);
    ALLOC(P->Acc, st_bytes);
    ALLOC(P->A, (size_t)P->nfin * P->geo.sa * es);
    ALLOC(P->B, (size_t)P->nfin * P->geo.sb * es);
    ALLOC(P->C, (size_t)P->nfout * P->geo.sb * es);
    ALLOC(P->tw, (size_t)n * es);
    P->twy = P->tw;
    P->twx = P->tw;
    if (P->geo.ny != n) ALLOC(P->twy, (size_t)P->geo.ny * es);
    if (P->geo.nx != n) {
        if (P->geo.nx == P->geo.ny) P->twx = P->twy;
        else ALLOC(P->twx, (size_t)P->geo.nx * es);
    }
    const int Kmax = std::max(K, std::max(P->geo.Kx, P->geo.Ky));
    const size_t nk2 = 3 * (size_t)Kmax * Kmax + 1;
    for (int i = 0; i < 2; ++i) {   // real factors; GPE: complex ones in the first pair
        ALLOC(P->Etab[i], nk2 * (gpe ? es : tsz));
        ALLOC(P->E2tab[i], nk2 * (gpe ? es : tsz));
    }
    ALLOC(P->red, sizeof(double) * (RED_BLOCKS + MAX_SHELLS + 8));
#undef ALLOC
    hipError_t e = hipMemsetAsync(P->U, 0, st_bytes, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) {
        fail(nullptr, PST_ERR_HIP, "initialising state failed: %s", hipGetErrorString(e));
        pst_plan_destroy(P);
        return PST_ERR_HIP;
    }
    s = p->precision == PST_FP64 ? upload_tables<double>(P) : upload_tables<float>(P);
    if (s != PST_OK) {
        g_create_err = P->err;
        pst_plan_destroy(P);
        return s;
    }
    *out = P;
    return PST_OK;
}

// shell width dk = the smallest a_i, and the shells a spectrum needs
static double shell_dk(const Geo& g) { return std::min(g.ax, std::min(g.ay, g.az)); }
static int shells_needed(const Geo& g) {
    if (!g.aniso && g.Kx == g.K && g.Ky == g.K) return (int)floor(sqrt(3.0) * g.K + 0.5) + 1;
    const double fx = g.ax * g.Kx, fy = g.ay * g.Ky, fz = g.az * g.K;
    return (int)floor(sqrt(fx * fx + fy * fy + fz * fz) / shell_dk(g) + 0.5) + 1;
}

extern "C" pst_status pst_query(const pst_plan* P, pst_info* info) {
    if (!P || !info) return PST_ERR_INVALID_ARG;
    info->n = P->p.n;
    info->kcut = P->geo.K;
    info->nx = P->geo.nx;
    info->ny = P->geo.ny;
    info->nz = P->geo.n;
    info->kcut_x = P->geo.Kx;
    info->kcut_y = P->geo.Ky;
    info->nshells = shells_needed(P->geo);
    info->ncomp = P->ncomp;
    info->modes_per_comp = (size_t)P->geo.sc;
    info->workspace_bytes = P->owned_bytes;
    for (int i = 0; i < 4; ++i) info->radices[i] = P->L->radices[i];
    info->tile_lines = P->L->tile_lines;
    info->steps_done = P->steps;
    return PST_OK;
}

// --------------------------------------------------------------- state I/O
static bool valid_field(const pst_plan* P, int field) {
    if (P->p.solver == PST_GPE) return field == PST_FIELD_PSI;
    return field == PST_FIELD_U || (field == PST_FIELD_B && P->p.solver == PST_MHD) ||
           (field == PST_FIELD_THETA && P->p.solver == PST_BOUSSINESQ);
}
// first state component and component count of a field
static int field_c0(int field) { return field == PST_FIELD_U || field == PST_FIELD_PSI ? 0 : 3; }
static int field_nc(int field) { return field == PST_FIELD_THETA || field == PST_FIELD_PSI ? 1 : 3; }
// the fields of the state, in component order
static int state_fields(const pst_plan* P, int* f) {
    if (P->p.solver == PST_GPE) {
        f[0] = PST_FIELD_PSI;
        return 1;
    }
    f[0] = PST_FIELD_U;
    if (P->p.solver == PST_MHD) f[1] = PST_FIELD_B;
    else if (P->p.solver == PST_BOUSSINESQ) f[1] = PST_FIELD_THETA;
    else return 1;
    return 2;
}

template <typename T>
static void launch_gather(pst_plan* P, const void* abi, void* st, int nc) {
    KTimer tm(P, PST_K_OTHER);
    hipLaunchKernelGGL((k_gather<T>), dim3(grid_for(nc * P->geo.sc)), dim3(256), 0, P->stream, (const cx<T>*)abi,
                       (cx<T>*)st, P->geo, nc);
}
template <typename T>
static void launch_scatter(pst_plan* P, const void* st, void* abi, int ncomp) {
    KTimer tm(P, PST_K_OTHER);
    const int64_t tot = (int64_t)abi_spec_bytes(P, ncomp) / (int64_t)P->esz;
    hipLaunchKernelGGL((k_scatter<T>), dim3(grid_for(tot)), dim3(256), 0, P->stream, (const cx<T>*)st,
                       (cx<T>*)abi, P->geo, ncomp);
}

static void gather(pst_plan* P, const void* abi, void* st, int nc) {
    if (P->p.precision == PST_FP64) launch_gather<double>(P, abi, st, nc);
    else launch_gather<float>(P, abi, st, nc);
}
static void scatter(pst_plan* P, const void* st, void* abi, int ncomp) {
    if (P->p.precision == PST_FP64) launch_scatter<double>(P, st, abi, ncomp);
    else launch_scatter<float>(P, st, abi, ncomp);
}

extern "C" pst_status pst_set_state(pst_plan* P, int field, int space, const void* src, int mem) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!src) return fail(P, PST_ERR_INVALID_ARG, "src is NULL");
    if (!valid_field(P, field)) return fail(P, PST_ERR_INVALID_ARG, "field %d invalid for this solver", field);
    if (space != PST_SPACE_PHYS && space != PST_SPACE_SPEC) return fail(P, PST_ERR_INVALID_ARG, "space %d", space);
    if (mem != PST_MEM_HOST && mem != PST_MEM_DEVICE) return fail(P, PST_ERR_INVALID_ARG, "mem %d", mem);
    const int nc = field_nc(field);
    const size_t spec = abi_spec_bytes(P, nc);
    // physical data: real, or complex for the GPE wavefunction
    const size_t phys = nc * phys_points(P) * (P->geo.full ? P->esz : P->esz / 2);
    // layout of the scratch: [spectral (nc comps)] [physical staging if needed]
    const size_t need = spec + ((space == PST_SPACE_PHYS && mem == PST_MEM_HOST) ? phys : 0);
    pst_status s = ensure_abi(P, need);
    if (s) return s;
    char* spec_buf = (char*)P->abi;
    if (space == PST_SPACE_SPEC) {
        if (mem == PST_MEM_HOST) {
            HIPCHK(P, hipMemcpyAsync(spec_buf, src, spec, hipMemcpyHostToDevice, P->stream));
        } else {
            HIPCHK(P, hipMemcpyAsync(spec_buf, src, spec, hipMemcpyDeviceToDevice, P->stream));
        }
    } else {
        const void* phys_dev = src;
        if (mem == PST_MEM_HOST) {
            HIPCHK(P, hipMemcpyAsync(spec_buf + spec, src, phys, hipMemcpyHostToDevice, P->stream));
            phys_dev = spec_buf + spec;
        }
        if (P->geo.full) fft3_c2c(P, phys_dev, spec_buf, nc, 0);
        else fft3_r2c(P, phys_dev, spec_buf, nc);
        if ((s = check_launch(P, "forward transform"))) return s;
    }
    char* st = (char*)P->U + (size_t)field_c0(field) * P->geo.sc * P->esz;
    gather(P, spec_buf, st, nc);
    if ((s = check_launch(P, "gather"))) return s;
    if (mem == PST_MEM_HOST) HIPCHK(P, hipStreamSynchronize(P->stream));
    P->steps = 0;
    return PST_OK;
}

extern "C" pst_status pst_get_state(pst_plan* P, int field, int space, void* dst, int mem) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!dst) return fail(P, PST_ERR_INVALID_ARG, "dst is NULL");
    if (!valid_field(P, field)) return fail(P, PST_ERR_INVALID_ARG, "field %d invalid for this solver", field);
    if (space != PST_SPACE_PHYS && space != PST_SPACE_SPEC) return fail(P, PST_ERR_INVALID_ARG, "space %d", space);
    if (mem != PST_MEM_HOST && mem != PST_MEM_DEVICE) return fail(P, PST_ERR_INVALID_ARG, "mem %d", mem);
    const int nc = field_nc(field);
    const size_t spec = abi_spec_bytes(P, nc);
    const size_t phys = nc * phys_points(P) * (P->geo.full ? P->esz : P->esz / 2);
    // scratch: [spectral] [c2r workspace (spectral)] [physical staging]
    const size_t need = space == PST_SPACE_SPEC ? spec : 2 * spec + (mem == PST_MEM_HOST ? phys : 0);
    pst_status s = ensure_abi(P, need);
    if (s) return s;
    char* spec_buf = (char*)P->abi;
    const char* st = (const char*)P->U + (size_t)field_c0(field) * P->geo.sc * P->esz;
    if (space == PST_SPACE_SPEC) {
        void* target = mem == PST_MEM_DEVICE ? dst : (void*)spec_buf;
        scatter(P, st, target, nc);
        if ((s = check_launch(P, "scatter"))) return s;
        if (mem == PST_MEM_HOST) {
            HIPCHK(P, hipMemcpyAsync(dst, spec_buf, spec, hipMemcpyDeviceToHost, P->stream));
            HIPCHK(P, hipStreamSynchronize(P->stream));
        }
    } else {
        scatter(P, st, spec_buf, nc);
        void* target = mem == PST_MEM_DEVICE ? dst : (void*)(spec_buf + 2 * spec);
        if (P->geo.full) fft3_c2c(P, spec_buf, target, nc, 1);
        else fft3_c2r(P, spec_buf, target, nc, spec_buf + spec);
        if ((s = check_launch(P, "backward transform"))) return s;
        if (mem == PST_MEM_HOST) {
            HIPCHK(P, hipMemcpyAsync(dst, target, phys, hipMemcpyDeviceToHost, P->stream));
            HIPCHK(P, hipStreamSynchronize(P->stream));
        }
    }
    return PST_OK;
}

// forcing: keep the box |k_i| <= kf that holds every nonzero mode
template <typename T>
static pst_status set_forcing_t(pst_plan* P, const cx<T>* h /*host ABI layout*/) {
    const Geo& g = P->geo;
    const int nx = g.nx, ny = g.ny, nz = g.n, nxh = nx / 2 + 1;
    // element (c, z, y, x) of the ABI layout
    auto at = [&](int c, int z, int y, int x) { return h[(((size_t)c * nz + z) * ny + y) * nxh + x]; };
    int kf = -1;
    for (int c = 0; c < 3; ++c)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nxh; ++x) {
                    const cx<T> v = at(c, z, y, x);
                    if (v.x == T(0) && v.y == T(0)) continue;
                    const int ky = k_of_pos(y, ny), kz = k_of_pos(z, nz);
                    if (x > g.Kx || abs(ky) > g.Ky || abs(kz) > g.K) continue;  // dealiased away
                    int m = x;
                    if (abs(ky) > m) m = abs(ky);
                    if (abs(kz) > m) m = abs(kz);
                    if (m > kf) kf = m;
                }
    if (P->force) {
        hipStreamSynchronize(P->stream);
        hipFree(P->force);
        P->force = nullptr;
    }
    P->kf = -1;
    if (kf < 0) return PST_OK;
    const int w = 2 * kf + 1;
    const size_t fs = (size_t)(kf + 1) * w * w;
    std::vector<cx<T>> box(3 * fs);
    for (int c = 0; c < 3; ++c)
        for (int kx = 0; kx <= kf; ++kx)
            for (int ky = -kf; ky <= kf; ++ky)
                for (int kz = -kf; kz <= kf; ++kz) {
                    cx<T> v = {T(0), T(0)};
                    if (kx <= g.Kx && abs(ky) <= g.Ky && abs(kz) <= g.K) {   // kept on every axis
                        const int y = (ky + ny) % ny, z = (kz + nz) % nz;
                        v = at(c, z, y, kx);
                        if (kx == 0) {  // Hermitian part, as for the state
                            const cx<T> m = at(c, (nz - z) % nz, (ny - y) % ny, 0);
                            v = {T(0.5) * (v.x + m.x), T(0.5) * (v.y - m.y)};
                        }
                    }
                    box[c * fs + ((size_t)kx * w + (ky + kf)) * w + (kz + kf)] = v;
                }
    void* d = nullptr;
    if (hipMalloc(&d, sizeof(cx<T>) * 3 * fs) != hipSuccess) {
        (void)hipGetLastError();
        return fail(P, PST_ERR_OOM, "forcing box allocation failed");
    }
    if (hipMemcpy(d, box.data(), sizeof(cx<T>) * 3 * fs, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(d);
        return fail(P, PST_ERR_HIP, "forcing upload failed");
    }
    P->force = d;
    P->kf = kf;
    return PST_OK;
}

extern "C" pst_status pst_set_forcing(pst_plan* P, const void* fhat, int mem) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (P->p.solver == PST_MHD || P->p.solver == PST_GPE)
        return fail(P, PST_ERR_INVALID_ARG, "forcing is defined for the Navier-Stokes and Boussinesq solvers only");
    if (mem != PST_MEM_HOST && mem != PST_MEM_DEVICE) return fail(P, PST_ERR_INVALID_ARG, "mem %d", mem);
    const size_t bytes = abi_spec_bytes(P, 3);
    std::vector<char> host;
    const void* h = fhat;
    if (fhat && mem == PST_MEM_DEVICE) {
        host.resize(bytes);
        HIPCHK(P, hipStreamSynchronize(P->stream));
        HIPCHK(P, hipMemcpy(host.data(), fhat, bytes, hipMemcpyDeviceToHost));
        h = host.data();
    }
    if (!h) {
        if (P->force) {
            hipStreamSynchronize(P->stream);
            hipFree(P->force);
            P->force = nullptr;
        }
        P->kf = -1;
        return PST_OK;
    }
    return P->p.precision == PST_FP64 ? set_forcing_t<double>(P, (const cx<double>*)h)
                                      : set_forcing_t<float>(P, (const cx<float>*)h);
}

// --------------------------------------------------------------- rhs / step
static pst_status run_rhs_passes(pst_plan* P, const void* state, int mode, void* rhs_out) {
    pst_status s;
    P->L->zinv(P, state);
    if ((s = check_launch(P, "zinv"))) return s;
    P->Ly->yinv(P);
    if ((s = check_launch(P, "yinv"))) return s;
    P->Lx->xpass(P);
    if ((s = check_launch(P, "xpass"))) return s;
    P->Ly->yfwd(P);
    if ((s = check_launch(P, "yfwd"))) return s;
    P->L->zfwd(P, mode, rhs_out);
    return check_launch(P, "zfwd");
}

extern "C" pst_status pst_rhs(pst_plan* P, const void* state_dev, void* rhs_dev) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!state_dev || !rhs_dev) return fail(P, PST_ERR_INVALID_ARG, "NULL buffer");
    const size_t spec = abi_spec_bytes(P, P->ncomp);
    const size_t cbytes = (size_t)P->ncomp * P->geo.sc * P->esz;
    pst_status s = ensure_abi(P, 2 * cbytes);
    if (s) return s;
    char* cst = (char*)P->abi;          // compact copy of the input state
    char* crhs = cst + cbytes;          // compact rhs
    (void)spec;
    int fl[2];
    const int nfl = state_fields(P, fl);
    for (int i = 0; i < nfl; ++i) {
        const int c0 = field_c0(fl[i]);
        const char* src = (const char*)state_dev + (size_t)c0 * abi_spec_bytes(P, 1);
        gather(P, src, cst + (size_t)c0 * P->geo.sc * P->esz, field_nc(fl[i]));
    }
    if ((s = check_launch(P, "gather"))) return s;
    if ((s = run_rhs_passes(P, cst, Z_RHS, crhs))) return s;
    scatter(P, crhs, rhs_dev, P->ncomp);
    return check_launch(P, "scatter");
}

extern "C" pst_status pst_step(pst_plan* P, int nsteps) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (nsteps < 0) return fail(P, PST_ERR_INVALID_ARG, "nsteps < 0");
    static const int rk4[4] = {Z_RK4_0, Z_RK4_1, Z_RK4_2, Z_RK4_3};
    static const int rk2[2] = {Z_RK2_0, Z_RK2_1};
    const int ns = P->p.rk_order == 4 ? 4 : 2;
    const int* modes = P->p.rk_order == 4 ? rk4 : rk2;
    for (int it = 0; it < nsteps; ++it) {
        for (int st = 0; st < ns; ++st) {
            pst_status s = run_rhs_passes(P, st == 0 ? P->U : P->V, modes[st], nullptr);
            if (s) return s;
        }
        P->steps++;
    }
    return PST_OK;
}

// --------------------------------------------------------------- diagnostics
template <typename T>
static void launch_energy(pst_plan* P, int c0, int nc, double* out, int k2w, double scale) {
    KTimer tm(P, PST_K_OTHER);
    hipLaunchKernelGGL((k_energy_part<T>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, P->stream, (const cx<T>*)P->U,
                       P->geo, c0, nc, P->red, k2w);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(RED_THREADS), 0, P->stream, P->red, RED_BLOCKS, out, scale);
}
static void launch_energy_p(pst_plan* P, int c0, int nc, double* out, int k2w, double scale) {
    if (P->p.precision == PST_FP64) launch_energy<double>(P, c0, nc, out, k2w, scale);
    else launch_energy<float>(P, c0, nc, out, k2w, scale);
}

// energy (k2w = 0) or enstrophy (k2w = 1) of u and b
static pst_status quadratic_diag(pst_plan* P, double out[2], int k2w, const char* what) {
    if (!P || !out) return P ? fail(P, PST_ERR_INVALID_ARG, "out is NULL") : PST_ERR_INVALID_ARG;
    double* res = P->red + RED_BLOCKS + MAX_SHELLS;
    int fl[2];
    int nfl = state_fields(P, fl);
    if (P->p.solver == PST_GPE) {
        // energy: particle number and kinetic energy alpha sum |k|^2 |psi|^2;
        // enstrophy: sum |k|^2 |psi|^2 alone
        launch_energy_p(P, 0, 1, res, k2w, 1.0);
        if (!k2w) launch_energy_p(P, 0, 1, res + 1, 1, P->p.alpha);
        nfl = k2w ? 1 : 2;
    } else {
        for (int i = 0; i < nfl; ++i) launch_energy_p(P, field_c0(fl[i]), field_nc(fl[i]), res + i, k2w, 0.5);
    }
    pst_status s = check_launch(P, what);
    if (s) return s;
    double h[2] = {0.0, 0.0};
    HIPCHK(P, hipMemcpyAsync(h, res, sizeof(double) * nfl, hipMemcpyDeviceToHost, P->stream));
    HIPCHK(P, hipStreamSynchronize(P->stream));
    out[0] = h[0];
    out[1] = nfl == 2 ? h[1] : 0.0;
    if (!isfinite(out[0]) || !isfinite(out[1])) return fail(P, PST_ERR_NONFINITE, "%s is not finite", what);
    return PST_OK;
}

// ------------------------------------------------------------ projection of spectral fields
// In place on the ABI spectral layout [ngroups][3][nz][ny][nx/2+1]: every mode
// outside the dealiasing cube is zeroed, the others are projected onto
// divergence-free fields, v - k (k . v) / |k|^2 (k = 0 kept).
template <typename T>
__global__ void k_project_abi(cx<T>* __restrict__ spec, Geo g, int ngroups) {
    const int nx = g.nx, ny = g.ny, nz = g.n, nxh = nx / 2 + 1;
    const int64_t per = (int64_t)nz * ny * nxh, total = (int64_t)ngroups * per;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t grp = i / per, r0 = i % per;
        const int kx = (int)(r0 % nxh);
        const int iy = (int)((r0 / nxh) % ny), iz = (int)(r0 / ((int64_t)nxh * ny));
        const int ky = k_of_pos(iy, ny), kz = k_of_pos(iz, nz);
        cx<T>* v = spec + grp * 3 * per + r0;
        cx<T> a = v[0], b = v[per], c = v[2 * per];
        if (kx > g.Kx || ky > g.Ky || -ky > g.Ky || kz > g.K || -kz > g.K) {
            a = b = c = {T(0), T(0)};
        } else if (kx != 0 || ky != 0 || kz != 0) {
            const T fx = T(g.ax) * T(kx), fy = T(g.ay) * T(ky), fz = T(g.az) * T(kz);
            const T ik2 = T(1) / (fx * fx + fy * fy + fz * fz);
            const T kr = (fx * a.x + fy * b.x + fz * c.x) * ik2, ki = (fx * a.y + fy * b.y + fz * c.y) * ik2;
            a = {a.x - fx * kr, a.y - fx * ki};
            b = {b.x - fy * kr, b.y - fy * ki};
            c = {c.x - fz * kr, c.y - fz * ki};
        }
        v[0] = a;
        v[per] = b;
        v[2 * per] = c;
    }
}

// Per group: partial sums of 1/2 w |v|^2 and 1/2 w |k|^2 |v|^2 (w = 1 on the
// kx = 0 and kx = nx/2 planes, else 2) over blockIdx.x's share, fixed order.
constexpr int PROJ_BLOCKS = 64;
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_quad_abi_part(const cx<T>* __restrict__ spec, Geo g,
                                                               double* __restrict__ part) {
    __shared__ double se[RED_THREADS], sz[RED_THREADS];
    const int nx = g.nx, ny = g.ny, nz = g.n, nxh = nx / 2 + 1;
    const int64_t per = (int64_t)nz * ny * nxh;
    const cx<T>* base = spec + (int64_t)blockIdx.y * 3 * per;
    double e = 0.0, z = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (int64_t)gridDim.x * blockDim.x) {
        const int kx = (int)(i % nxh);
        const int ky = k_of_pos((int)((i / nxh) % ny), ny), kz = k_of_pos((int)(i / ((int64_t)nxh * ny)), nz);
        const double w = (kx == 0 || 2 * kx == nx) ? 0.5 : 1.0;
        double q = 0.0;
        for (int c = 0; c < 3; ++c) {
            const cx<T> v = base[c * per + i];
            q += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
        const double fx = g.ax * kx, fy = g.ay * ky, fz = g.az * kz;
        e += w * q;
        z += w * (fx * fx + fy * fy + fz * fz) * q;
    }
    se[threadIdx.x] = e;
    sz[threadIdx.x] = z;
    __syncthreads();
    for (int h = RED_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            se[threadIdx.x] += se[threadIdx.x + h];
            sz[threadIdx.x] += sz[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * ((int64_t)blockIdx.y * PROJ_BLOCKS + blockIdx.x)] = se[0];
        part[2 * ((int64_t)blockIdx.y * PROJ_BLOCKS + blockIdx.x) + 1] = sz[0];
    }
}

__global__ void k_quad_abi_final(const double* __restrict__ part, double* __restrict__ out) {
    // one thread per (group, quantity): the PROJ_BLOCKS partials in order
    const int grp = blockIdx.x, q = threadIdx.x;
    if (q > 1) return;
    double s = 0.0;
    for (int b = 0; b < PROJ_BLOCKS; ++b) s += part[2 * (grp * PROJ_BLOCKS + b) + q];
    out[2 * grp + q] = s;
}

template <typename T>
static void launch_project(pst_plan* P, void* spec, int ngroups, double* part, double* res) {
    KTimer tm(P, PST_K_OTHER);
    const int64_t tot = (int64_t)ngroups * (abi_spec_bytes(P, 1) / P->esz);
    hipLaunchKernelGGL((k_project_abi<T>), dim3(grid_for(tot)), dim3(256), 0, P->stream, (cx<T>*)spec, P->geo, ngroups);
    if (part) {
        hipLaunchKernelGGL((k_quad_abi_part<T>), dim3(PROJ_BLOCKS, ngroups), dim3(RED_THREADS), 0, P->stream,
                           (const cx<T>*)spec, P->geo, part);
        hipLaunchKernelGGL(k_quad_abi_final, dim3(ngroups), dim3(64), 0, P->stream, part, res);
    }
}

extern "C" pst_status pst_project(pst_plan* P, void* spec_dev, int ngroups, double* energy, double* enstrophy) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!spec_dev) return fail(P, PST_ERR_INVALID_ARG, "NULL buffer");
    if (ngroups < 1) return fail(P, PST_ERR_INVALID_ARG, "ngroups < 1");
    if (P->geo.full) return fail(P, PST_ERR_UNSUPPORTED, "projection of a complex field");
    const bool diag = energy || enstrophy;
    double* part = nullptr;
    if (diag) {
        // partials and results in the plan's spectral scratch (stream-ordered
        // after any earlier call that used it; grown with a synchronisation)
        const size_t need = sizeof(double) * (size_t)ngroups * (2 * PROJ_BLOCKS + 2);
        pst_status s = ensure_abi(P, need);
        if (s) return s;
        part = (double*)P->abi;
    }
    double* res = part ? part + 2 * (size_t)ngroups * PROJ_BLOCKS : nullptr;
    if (P->p.precision == PST_FP64) launch_project<double>(P, spec_dev, ngroups, part, res);
    else launch_project<float>(P, spec_dev, ngroups, part, res);
    pst_status s = check_launch(P, "project");
    if (s || !diag) return s;
    std::vector<double> h(2 * (size_t)ngroups);
    HIPCHK(P, hipMemcpyAsync(h.data(), res, sizeof(double) * h.size(), hipMemcpyDeviceToHost, P->stream));
    HIPCHK(P, hipStreamSynchronize(P->stream));
    for (int i = 0; i < ngroups; ++i) {
        if (energy) energy[i] = h[2 * i];
        if (enstrophy) enstrophy[i] = h[2 * i + 1];
        if (!isfinite(h[2 * i]) || !isfinite(h[2 * i + 1])) return fail(P, PST_ERR_NONFINITE, "group %d", i);
    }
    return PST_OK;
}

extern "C" pst_status pst_energy(pst_plan* P, double out[2]) { return quadratic_diag(P, out, 0, "energy"); }

extern "C" pst_status pst_enstrophy(pst_plan* P, double out[2]) { return quadratic_diag(P, out, 1, "enstrophy"); }

extern "C" pst_status pst_spectrum(pst_plan* P, int field, double* Ek, int nshells) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!Ek) return fail(P, PST_ERR_INVALID_ARG, "Ek is NULL");
    if (!valid_field(P, field)) return fail(P, PST_ERR_INVALID_ARG, "field %d", field);
    const int need = shells_needed(P->geo);
    if (nshells < need || nshells > MAX_SHELLS)
        return fail(P, PST_ERR_INVALID_ARG, "nshells must be in [%d, %d]", need, MAX_SHELLS);
    double* bins = P->red + RED_BLOCKS;
    {
        KTimer tm(P, PST_K_OTHER);
        const double dk = shell_dk(P->geo);
        if (P->p.precision == PST_FP64)
            hipLaunchKernelGGL((k_spectrum<double>), dim3(nshells), dim3(RED_THREADS), 0, P->stream,
                               (const cx<double>*)P->U, P->geo, field_c0(field), field_nc(field), bins, dk);
        else
            hipLaunchKernelGGL((k_spectrum<float>), dim3(nshells), dim3(RED_THREADS), 0, P->stream,
                               (const cx<float>*)P->U, P->geo, field_c0(field), field_nc(field), bins, dk);
    }
    pst_status s = check_launch(P, "spectrum");
    if (s) return s;
    HIPCHK(P, hipMemcpyAsync(Ek, bins, sizeof(double) * nshells, hipMemcpyDeviceToHost, P->stream));
    HIPCHK(P, hipStreamSynchronize(P->stream));
    for (int i = 0; i < nshells; ++i)
        if (!isfinite(Ek[i])) return fail(P, PST_ERR_NONFINITE, "spectrum is not finite");
    return PST_OK;
}

// --------------------------------------------------------------- transforms
extern "C" pst_status pst_fft_r2c(pst_plan* P, const void* in, void* out, int nfields) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!in || !out) return fail(P, PST_ERR_INVALID_ARG, "NULL buffer");
    if (nfields < 1) return fail(P, PST_ERR_INVALID_ARG, "nfields < 1");
    fft3_r2c(P, in, out, nfields);
    return check_launch(P, "fft_r2c");
}

extern "C" pst_status pst_fft_c2r(pst_plan* P, const void* in, void* out, int nfields) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!in || !out) return fail(P, PST_ERR_INVALID_ARG, "NULL buffer");
    if (nfields < 1) return fail(P, PST_ERR_INVALID_ARG, "nfields < 1");
    pst_status s = ensure_abi(P, abi_spec_bytes(P, nfields));
    if (s) return s;
    fft3_c2r(P, in, out, nfields, P->abi);
    return check_launch(P, "fft_c2r");
}

// --------------------------------------------------------------- timers
extern "C" pst_status pst_timer_read(pst_plan* P, double* ms, long long* count, int reset) {
    if (!P) return PST_ERR_INVALID_ARG;
    if (!(P->p.flags & PST_FLAG_TIMERS)) return fail(P, PST_ERR_UNSUPPORTED, "plan created without PST_FLAG_TIMERS");
    HIPCHK(P, hipStreamSynchronize(P->stream));
    drain_timers(P);
    for (int k = 0; k < PST_K_COUNT; ++k) {
        if (ms) ms[k] = P->t_ms[k];
        if (count) count[k] = P->t_cnt[k];
        if (reset) {
            P->t_ms[k] = 0.0;
            P->t_cnt[k] = 0;
        }
    }
    return PST_OK;
}
