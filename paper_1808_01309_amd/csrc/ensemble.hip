// Ensembles of independent Navier-Stokes runs of uneven grid sizes advanced
// together (host side; device code in ensemble_kernels.h).  Runs are grouped
// into classes of equal n; each class keeps its runs' buffers back to back.
// Ways to run an RK step (pst_ensemble_set_mode):
//   0 PERSISTENT + GRAPH  the persistent step kernel captured once in a HIP
//                         graph and replayed every step (default);
//   1 PERSISTENT          one launch per step: every block loops over the work
//                         units of all runs for each pass of every RK stage,
//                         with a device-wide barrier between passes;
//   2 BATCHED             one launch per (pass, class) covering all its runs;
//   3 SEQUENTIAL          one launch per (pass, run);
//   4 BATCHED + GRAPH     the batched launches of one step captured once in a
//                         HIP graph and replayed every step.
// The schedule variant (radix order x tile lines) is picked by timing the
// candidates (pst_ensemble_autotune) and cached.  FP32 only.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "ensemble_kernels.h"

namespace pst {
const EnsKernels* ens_kernels_v0();
const EnsKernels* ens_kernels_v1();
const EnsKernels* ens_kernels_v2();
const EnsKernels* ens_kernels_v3();
static const EnsKernels* ens_kernels(int v) {
    switch (v) {
        case 0: return ens_kernels_v0();
        case 1: return ens_kernels_v1();
        case 2: return ens_kernels_v2();
        default: return ens_kernels_v3();
    }
}

// Barrier words back to zero before every persistent step (a timed-out
// barrier leaves its counters part-way).  The timeout flag is not touched
// here: it is cleared by the host before and after each pst_ensemble_step, so
// a timeout in any step of a multi-step call is still reported.
__global__ void k_ens_reset_bar(unsigned* bar) {
    for (int i = threadIdx.x; i < ENS_BAR_WORDS; i += blockDim.x) bar[i] = 0u;
}
__global__ void k_ens_clear_err(int* err) {
    if (threadIdx.x == 0) err[0] = 0;
}

template <typename T>
__global__ void k_ens_energy(EnsClass<T> c, double* out) {
    // one block per run: E = 1/2 sum w |u|^2, fixed-order tree reduction
    __shared__ double sh[256];
    const int run = blockIdx.x;
    const cx<T>* U = c.U + run * c.s_st;
    const Geo& g = c.geo;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < g.sc; i += blockDim.x) {
        const double w = (i / ((int64_t)g.M * g.M)) == 0 ? 1.0 : 2.0;
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const cx<T> v = U[k * g.sc + i];
            s += (double)v.x * v.x + (double)v.y * v.y;
        }
        acc += w * s;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[run] = 0.5 * sh[0];
}

// energy and enstrophy of every run of a class (one block per run)
template <typename T>
__global__ void k_ens_diag(EnsClass<T> c, double* out_e, double* out_z) {
    __shared__ double se[256], sz[256];
    const int run = blockIdx.x;
    const cx<T>* U = c.U + run * c.s_st;
    const Geo& g = c.geo;
    double ae = 0.0, az = 0.0;
    for (int64_t i = threadIdx.x; i < g.sc; i += blockDim.x) {
        const int jz = (int)(i % g.M), jy = (int)((i / g.M) % g.M), kx = (int)(i / ((int64_t)g.M * g.M));
        const int ky = k_of_j(jy, g), kz = k_of_j(jz, g);
        const double w = kx == 0 ? 1.0 : 2.0, k2 = (double)(kx * kx + ky * ky + kz * kz);
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const cx<T> v = U[k * g.sc + i];
            s += (double)v.x * v.x + (double)v.y * v.y;
        }
        ae += w * s;
        az += w * k2 * s;
    }
    se[threadIdx.x] = ae;
    sz[threadIdx.x] = az;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            se[threadIdx.x] += se[threadIdx.x + w];
            sz[threadIdx.x] += sz[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_e[run] = 0.5 * se[0];
        out_z[run] = 0.5 * sz[0];
    }
}

// projection onto divergence-free fields of every run of a class (k = 0 kept)
template <typename T>
__global__ void k_ens_project(EnsClass<T> c) {
    const Geo& g = c.geo;
    const int64_t total = (int64_t)c.nruns * g.sc;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int run = (int)(t / g.sc);
        const int64_t i = t % g.sc;
        const int jz = (int)(i % g.M), jy = (int)((i / g.M) % g.M), kx = (int)(i / ((int64_t)g.M * g.M));
        const T fx = T(kx), fy = T(k_of_j(jy, g)), fz = T(k_of_j(jz, g));
        const T k2 = fx * fx + fy * fy + fz * fz;
        if (k2 == T(0)) continue;
        cx<T>* U = c.U + run * c.s_st + i;
        const cx<T> a = U[0], b = U[g.sc], d = U[2 * g.sc];
        const cx<T> kv = {(fx * a.x + fy * b.x + fz * d.x) / k2, (fx * a.y + fy * b.y + fz * d.y) / k2};
        U[0] = {a.x - fx * kv.x, a.y - fx * kv.y};
        U[g.sc] = {b.x - fy * kv.x, b.y - fy * kv.y};
        U[2 * g.sc] = {d.x - fz * kv.x, d.y - fz * kv.y};
    }
}

// per run: sum w |a - b|^2 and sum w |b|^2 (one block per run)
template <typename T>
__global__ void k_ens_dist(EnsClass<T> a, EnsClass<T> b, double* out) {
    __shared__ double sd[256], sb[256];
    const int run = blockIdx.x;
    const Geo& g = a.geo;
    const cx<T>* A = a.U + run * a.s_st;
    const cx<T>* Bv = b.U + run * b.s_st;
    double dd = 0.0, bb = 0.0;
    for (int64_t i = threadIdx.x; i < 3 * g.sc; i += blockDim.x) {
        const double w = ((i % g.sc) / ((int64_t)g.M * g.M)) == 0 ? 1.0 : 2.0;
        const cx<T> x = A[i], y = Bv[i];
        const double ex = (double)x.x - y.x, ey = (double)x.y - y.y;
        dd += w * (ex * ex + ey * ey);
        bb += w * ((double)y.x * y.x + (double)y.y * y.y);
    }
    sd[threadIdx.x] = dd;
    sb[threadIdx.x] = bb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sd[threadIdx.x] += sd[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * run] = sd[0];
        out[2 * run + 1] = sb[0];
    }
}

template <typename T>
__global__ void k_ens_gather(const cx<T>* __restrict__ abi, cx<T>* __restrict__ st, Geo g) {
    const int64_t total = 3 * g.sc;
    const int nxh = g.n / 2 + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / g.sc);
        int64_t r = i % g.sc;
        const int jz = (int)(r % g.M);
        r /= g.M;
        const int jy = (int)(r % g.M);
        const int kx = (int)(r / g.M);
        const int iy = (k_of_j(jy, g) + g.n) % g.n, iz = (k_of_j(jz, g) + g.n) % g.n;
        const cx<T>* a = abi + (int64_t)c * g.n * g.n * nxh;
        cx<T> v = a[((int64_t)iz * g.n + iy) * nxh + kx];
        if (kx == 0) {
            const cx<T> m = a[((int64_t)((g.n - iz) % g.n) * g.n + (g.n - iy) % g.n) * nxh];
            v = {T(0.5) * (v.x + m.x), T(0.5) * (v.y - m.y)};
        }
        st[i] = v;
    }
}

template <typename T>
__global__ void k_ens_scatter(const cx<T>* __restrict__ st, cx<T>* __restrict__ abi, Geo g) {
    const int nxh = g.n / 2 + 1;
    const int64_t per = (int64_t)g.n * g.n * nxh, total = 3 * per;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / per);
        int64_t r = i % per;
        const int kx = (int)(r % nxh);
        r /= nxh;
        const int ky = k_of_pos((int)(r % g.n), g.n), kz = k_of_pos((int)(r / g.n), g.n);
        cx<T> v = {T(0), T(0)};
        if (kx <= g.K && ky <= g.K && -ky <= g.K && kz <= g.K && -kz <= g.K) {
            const int jy = ky >= 0 ? ky : ky + g.M, jz = kz >= 0 ? kz : kz + g.M;
            v = st[(int64_t)c * g.sc + ((int64_t)kx * g.M + jy) * g.M + jz];
        }
        abi[i] = v;
    }
}


}  // namespace pst

using namespace pst;

struct EnsClassHost {
    int n;
    std::vector<int> runs;   // global run ids
    void *U, *V, *Acc, *A, *B, *C, *tw, *E, *E2;
    Geo geo;
};

struct pst_ensemble {
    pst_params p;
    hipStream_t stream;
    int nruns;
    std::vector<int> run_class, run_index;
    std::vector<EnsClassHost> cls;
    int mode;
    int var;                      // schedule variant of the persistent kernel
    int cvar[ENS_MAX_CLASSES];    // per class: the variant of its batched / sequential launches
    int grids[ENS_NVAR];
    EnsDesc<float> desc_host;     // last descriptor uploaded to desc_dev
    EnsDesc<float>* desc_dev;
    unsigned* bar;
    int* err;
    double* eout;
    void* scratch;
    size_t scratch_bytes;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_valid;
    long long spin_limit;         // polls of a device-wide barrier before it reports a timeout
    std::string msg;
    size_t owned;
};

static thread_local std::string g_ens_err;

static pst_status efail(pst_ensemble* E, pst_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (E) E->msg = buf;
    else g_ens_err = buf;
    return s;
}

// per_class: the work units of each class follow its own variant (the
// batched and sequential launches); else all follow the persistent kernel's.
static EnsDesc<float> make_desc(pst_ensemble* E, bool per_class) {
    EnsDesc<float> d;
    memset(&d, 0, sizeof d);
    d.ncls = (int)E->cls.size();
    for (int i = 0; i < d.ncls; ++i) {
        const EnsKernels* K = ens_kernels(per_class ? E->cvar[i] : E->var);
        const EnsClassHost& h = E->cls[i];
        EnsClass<float>& c = d.cls[i];
        c.geo = h.geo;
        c.nruns = (int)h.runs.size();
        c.U = (cx<float>*)h.U;
        c.V = (cx<float>*)h.V;
        c.Acc = (cx<float>*)h.Acc;
        c.A = (cx<float>*)h.A;
        c.B = (cx<float>*)h.B;
        c.C = (cx<float>*)h.C;
        c.s_st = 3 * h.geo.sc;
        c.s_a = 6 * h.geo.sa;
        c.s_b = 6 * h.geo.sb;
        c.s_c = 3 * h.geo.sb;
        c.tw = (const cx<float>*)h.tw;
        c.E = (const float*)h.E;
        c.E2 = (const float*)h.E2;
        K->units(h.geo, c.upr);
    }
    if (E->p.rk_order == 4) {
        d.nstages = 4;
        d.modes[0] = Z_RK4_0; d.modes[1] = Z_RK4_1; d.modes[2] = Z_RK4_2; d.modes[3] = Z_RK4_3;
    } else {
        d.nstages = 2;
        d.modes[0] = Z_RK2_0; d.modes[1] = Z_RK2_1;
    }
    d.h = (float)E->p.dt;
    d.bar = E->bar;
    d.err = E->err;
    d.spin_limit = E->spin_limit;
    return d;
}

// Blocks of the persistent kernel: as many as are co-resident on the device
// (the device-wide barrier needs every block running at once).
static int persistent_grid(const EnsKernels* K) {
    int dev = 0, ncu = 0, per = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, K->persistent, ENS_NT, 0) != hipSuccess) per = 1;
    if (per < 1) per = 1;
    return ncu * per;
}

static void launch_step(pst_ensemble* E) {
    const bool pers = E->mode == 0 || E->mode == 1;
    EnsDesc<float> d = make_desc(E, !pers);
    if (pers) {
        const EnsKernels* K = ens_kernels(E->var);
        // the descriptor only changes with the schedule: upload it when it does
        if (memcmp(&d, &E->desc_host, sizeof d) != 0) {
            E->desc_host = d;
            hipMemcpyAsync(E->desc_dev, &E->desc_host, sizeof d, hipMemcpyHostToDevice, E->stream);
        }
        hipLaunchKernelGGL(k_ens_reset_bar, dim3(1), dim3(64), 0, E->stream, E->bar);
        K->launch_persistent(E->desc_dev, E->grids[E->var], E->stream);
        return;
    }
    for (int s = 0; s < d.nstages; ++s)
        for (int pass = 0; pass < 5; ++pass)
            for (int c = 0; c < d.ncls; ++c) {
                const EnsKernels* K = ens_kernels(E->cvar[c]);
                if (E->mode == 2 || E->mode == 4) K->launch_pass(d.cls[c], pass, s > 0, d.modes[s], d.h, E->stream);
                else
                    for (int r = 0; r < d.cls[c].nruns; ++r)
                        K->launch_pass_run(d.cls[c], pass, s > 0, d.modes[s], d.h, r, E->stream);
            }
}

static void drop_graph(pst_ensemble* E) {
    if (E->graph_valid) {
        hipGraphExecDestroy(E->gexec);
        hipGraphDestroy(E->graph);
        E->graph_valid = false;
    }
}

template <typename T>
static pst_status ens_tables(pst_ensemble* E, EnsClassHost& h) {
    const int n = h.n, K = h.geo.K;
    std::vector<cx<T>> tw(n);
    for (int m = 0; m < n; ++m) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
        tw[m].x = (T)cosl(a);
        tw[m].y = (T)(-sinl(a));
    }
    const int nk2 = 3 * K * K + 1;
    std::vector<T> e(nk2), e2(nk2);
    for (int k2 = 0; k2 < nk2; ++k2) {
        const double v = exp(-E->p.nu * (double)k2 * E->p.dt * 0.5);
        e[k2] = (T)v;
        e2[k2] = (T)(v * v);
    }
    if (hipMemcpy(h.tw, tw.data(), sizeof(cx<T>) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h.E, e.data(), sizeof(T) * nk2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h.E2, e2.data(), sizeof(T) * nk2, hipMemcpyHostToDevice) != hipSuccess)
        return efail(E, PST_ERR_HIP, "uploading tables failed");
    return PST_OK;
}

extern "C" void pst_ensemble_destroy(pst_ensemble* E) {
    if (!E) return;
    hipStreamSynchronize(E->stream);
    drop_graph(E);
    for (auto& c : E->cls)
        for (void* p : {c.U, c.V, c.Acc, c.A, c.B, c.C, c.tw, c.E, c.E2})
            if (p) hipFree(p);
    for (void* p : {(void*)E->desc_dev, (void*)E->bar, (void*)E->err, (void*)E->eout, E->scratch})
        if (p) hipFree(p);
    delete E;
}

extern "C" const char* pst_ensemble_last_error(const pst_ensemble* E) { return E ? E->msg.c_str() : g_ens_err.c_str(); }

extern "C" pst_status pst_ensemble_create(int nruns, const int* n, const pst_params* common, void* hip_stream,
                                          pst_ensemble** out) {
    g_ens_err.clear();
    if (!out) return efail(nullptr, PST_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!n || !common || nruns < 1) return efail(nullptr, PST_ERR_INVALID_ARG, "need nruns >= 1, sizes and params");
    if (common->solver != PST_NS) return efail(nullptr, PST_ERR_UNSUPPORTED, "ensembles run the Navier-Stokes solver");
    if (common->precision == PST_FP64) return efail(nullptr, PST_ERR_UNSUPPORTED, "ensembles run in FP32");
    if (common->precision != PST_FP32) return efail(nullptr, PST_ERR_INVALID_ARG, "precision %d", common->precision);
    if (common->rk_order != 2 && common->rk_order != 4)
        return efail(nullptr, PST_ERR_INVALID_ARG, "rk_order %d", common->rk_order);
    if (!(common->dt > 0.0) || !(common->nu >= 0.0) || !isfinite(common->dt) || !isfinite(common->nu))
        return efail(nullptr, PST_ERR_INVALID_ARG, "dt must be > 0 and nu >= 0");
    if (common->flags != 0) return efail(nullptr, PST_ERR_UNSUPPORTED, "flags are not supported for ensembles");
    if (common->dealias != PST_DEALIAS_CUBE)
        return efail(nullptr, PST_ERR_UNSUPPORTED, "ensembles use the cube truncation");
    // classes in descending n: the persistent kernel hands out the most
    // expensive work units first
    std::map<int, int, std::greater<int>> cls_of;
    for (int r = 0; r < nruns; ++r) {
        if (!ens_supported_n(n[r])) return efail(nullptr, PST_ERR_UNSUPPORTED_N, "run %d: n = %d", r, n[r]);
        if (!cls_of.count(n[r])) cls_of[n[r]] = 0;
    }
    if ((int)cls_of.size() > ENS_MAX_CLASSES) return efail(nullptr, PST_ERR_UNSUPPORTED, "too many distinct sizes");
    pst_ensemble* E = new pst_ensemble();
    E->p = *common;
    E->stream = (hipStream_t)hip_stream;
    E->nruns = nruns;
    E->mode = 0;
    E->graph_valid = false;
    E->spin_limit = 1ll << 22;
    memset(&E->desc_host, 0xff, sizeof E->desc_host);
    int ci = 0;
    for (auto& kv : cls_of) {
        kv.second = ci++;
        EnsClassHost h{};
        h.n = kv.first;
        const int nn = h.n, K = (nn + 2) / 3 - 1;
        h.geo = make_geo(nn, nn, nn, K, K, K, 1.0, 1.0, 1.0, 0);
        E->cls.push_back(h);
    }
    E->run_class.resize(nruns);
    E->run_index.resize(nruns);
    for (int r = 0; r < nruns; ++r) {
        const int c = cls_of[n[r]];
        E->run_class[r] = c;
        E->run_index[r] = (int)E->cls[c].runs.size();
        E->cls[c].runs.push_back(r);
    }
    const size_t es = 8, ts = 4;
    auto alloc = [&](void** p, size_t bytes) -> bool {
        if (hipMalloc(p, bytes) != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return false;
        }
        E->owned += bytes;
        return true;
    };
    bool ok = true;
    size_t maxspec = 0;
    for (auto& h : E->cls) {
        const size_t R = h.runs.size();
        const Geo& g = h.geo;
        const int nk2 = 3 * g.K * g.K + 1;
        ok = ok && alloc(&h.U, R * 3 * g.sc * es) && alloc(&h.V, R * 3 * g.sc * es) && alloc(&h.Acc, R * 3 * g.sc * es) &&
             alloc(&h.A, R * 6 * g.sa * es) && alloc(&h.B, R * 6 * g.sb * es) && alloc(&h.C, R * 3 * g.sb * es) &&
             alloc(&h.tw, h.n * es) && alloc(&h.E, nk2 * ts) && alloc(&h.E2, nk2 * ts);
        maxspec = std::max(maxspec, (size_t)3 * h.n * h.n * (h.n / 2 + 1) * es);
        if (!ok) break;
    }
    ok = ok && alloc((void**)&E->desc_dev, sizeof(EnsDesc<float>)) && alloc((void**)&E->bar, sizeof(unsigned) * ENS_BAR_WORDS) && alloc((void**)&E->err, 64) && alloc((void**)&E->eout, sizeof(double) * 2 * nruns) &&
         alloc(&E->scratch, maxspec);
    E->scratch_bytes = maxspec;
    if (!ok) {
        g_ens_err = "device allocation failed";
        pst_ensemble_destroy(E);
        return PST_ERR_OOM;
    }
    for (auto& h : E->cls) {
        hipMemsetAsync(h.U, 0, h.runs.size() * 3 * h.geo.sc * es, E->stream);
        pst_status s = ens_tables<float>(E, h);
        if (s) {
            g_ens_err = E->msg;
            pst_ensemble_destroy(E);
            return s;
        }
    }
    hipLaunchKernelGGL(k_ens_reset_bar, dim3(1), dim3(64), 0, E->stream, E->bar);
    hipLaunchKernelGGL(k_ens_clear_err, dim3(1), dim3(64), 0, E->stream, E->err);
    E->var = 0;
    for (int c = 0; c < ENS_MAX_CLASSES; ++c) E->cvar[c] = 0;
    for (int v = 0; v < ENS_NVAR; ++v) E->grids[v] = persistent_grid(ens_kernels(v));
    if (hipStreamSynchronize(E->stream) != hipSuccess) {
        g_ens_err = "initialisation failed";
        pst_ensemble_destroy(E);
        return PST_ERR_HIP;
    }
    *out = E;
    return PST_OK;
}

extern "C" pst_status pst_ensemble_set_state(pst_ensemble* E, int run, const void* uhat, int mem) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (run < 0 || run >= E->nruns || !uhat) return efail(E, PST_ERR_INVALID_ARG, "run %d / NULL input", run);
    if (mem != PST_MEM_HOST && mem != PST_MEM_DEVICE) return efail(E, PST_ERR_INVALID_ARG, "mem %d", mem);
    EnsClassHost& h = E->cls[E->run_class[run]];
    const size_t es = 8;
    const size_t bytes = (size_t)3 * h.n * h.n * (h.n / 2 + 1) * es;
    if (hipMemcpyAsync(E->scratch, uhat, bytes, mem == PST_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                       E->stream) != hipSuccess)
        return efail(E, PST_ERR_HIP, "copy failed");
    const size_t off = (size_t)E->run_index[run] * 3 * h.geo.sc * es;
    hipLaunchKernelGGL(k_ens_gather<float>, dim3(256), dim3(256), 0, E->stream, (const cx<float>*)E->scratch,
                           (cx<float>*)((char*)h.U + off), h.geo);
    if (hipGetLastError() != hipSuccess) return efail(E, PST_ERR_HIP, "gather launch failed");
    if (mem == PST_MEM_HOST && hipStreamSynchronize(E->stream) != hipSuccess) return efail(E, PST_ERR_HIP, "sync failed");
    return PST_OK;
}

extern "C" pst_status pst_ensemble_get_state(pst_ensemble* E, int run, void* uhat, int mem) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (run < 0 || run >= E->nruns || !uhat) return efail(E, PST_ERR_INVALID_ARG, "run %d / NULL output", run);
    if (mem != PST_MEM_HOST && mem != PST_MEM_DEVICE) return efail(E, PST_ERR_INVALID_ARG, "mem %d", mem);
    EnsClassHost& h = E->cls[E->run_class[run]];
    const size_t es = 8;
    const size_t bytes = (size_t)3 * h.n * h.n * (h.n / 2 + 1) * es;
    const size_t off = (size_t)E->run_index[run] * 3 * h.geo.sc * es;
    void* target = mem == PST_MEM_DEVICE ? uhat : E->scratch;
    hipLaunchKernelGGL(k_ens_scatter<float>, dim3(256), dim3(256), 0, E->stream,
                           (const cx<float>*)((char*)h.U + off), (cx<float>*)target, h.geo);
    if (hipGetLastError() != hipSuccess) return efail(E, PST_ERR_HIP, "scatter launch failed");
    if (mem == PST_MEM_HOST) {
        if (hipMemcpyAsync(uhat, E->scratch, bytes, hipMemcpyDeviceToHost, E->stream) != hipSuccess ||
            hipStreamSynchronize(E->stream) != hipSuccess)
            return efail(E, PST_ERR_HIP, "copy failed");
    }
    return PST_OK;
}

// Read the timeout flag of the persistent steps enqueued since it was last
// cleared, then clear it for the next call.
static pst_status check_err_flag(pst_ensemble* E) {
    int err = 0;
    if (hipMemcpyAsync(&err, E->err, sizeof(int), hipMemcpyDeviceToHost, E->stream) != hipSuccess ||
        hipStreamSynchronize(E->stream) != hipSuccess)
        return efail(E, PST_ERR_HIP, "reading the barrier flag failed");
    hipLaunchKernelGGL(k_ens_clear_err, dim3(1), dim3(64), 0, E->stream, E->err);
    if (err) return efail(E, PST_ERR_HIP, "persistent step: device-wide barrier timed out (grid not co-resident?)");
    return PST_OK;
}

extern "C" pst_status pst_ensemble_set_spin_limit(pst_ensemble* E, long long polls) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (polls < 0) return efail(E, PST_ERR_INVALID_ARG, "spin limit %lld < 0", polls);
    drop_graph(E);   // a captured step holds the old descriptor upload
    E->spin_limit = polls;
    return PST_OK;
}

extern "C" pst_status pst_ensemble_set_mode(pst_ensemble* E, int mode) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (mode < 0 || mode > 4) return efail(E, PST_ERR_INVALID_ARG, "mode %d", mode);
    drop_graph(E);
    E->mode = mode;
    return PST_OK;
}

extern "C" pst_status pst_ensemble_get_mode(const pst_ensemble* E, int* mode) {
    if (!E || !mode) return PST_ERR_INVALID_ARG;
    *mode = E->mode;
    return PST_OK;
}

extern "C" pst_status pst_ensemble_step(pst_ensemble* E, int nsteps) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (nsteps < 0) return efail(E, PST_ERR_INVALID_ARG, "nsteps < 0");
    if (nsteps == 0) return PST_OK;
    // the timeout flag starts clear (outside any captured graph); every step of
    // this call leaves it set if one of its barriers timed out, and the
    // persistent kernel returns at once while it is set
    if (E->mode <= 1) hipLaunchKernelGGL(k_ens_clear_err, dim3(1), dim3(64), 0, E->stream, E->err);
    if (E->mode == 0 || E->mode == 4) {  // one step's launches replayed from a captured graph
        if (!E->graph_valid) {
            hipStream_t cs = nullptr;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
                return efail(E, PST_ERR_HIP, "stream creation failed");
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipStream_t keep = E->stream;
                E->stream = cs;
                launch_step(E);
                E->stream = keep;
                e = hipStreamEndCapture(cs, &E->graph);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&E->gexec, E->graph, nullptr, nullptr, 0);
            hipStreamDestroy(cs);
            if (e != hipSuccess) return efail(E, PST_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
            E->graph_valid = true;
        }
        for (int i = 0; i < nsteps; ++i)
            if (hipGraphLaunch(E->gexec, E->stream) != hipSuccess) return efail(E, PST_ERR_HIP, "graph launch failed");
    } else {
        for (int i = 0; i < nsteps; ++i) launch_step(E);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return efail(E, PST_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
    }
    if (E->mode <= 1) return check_err_flag(E);
    return PST_OK;
}

extern "C" pst_status pst_ensemble_energy(pst_ensemble* E, double* per_run) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (!per_run) return efail(E, PST_ERR_INVALID_ARG, "NULL output");
    EnsDesc<float> d = make_desc(E, false);
    for (int c = 0; c < d.ncls; ++c) {
        const EnsClassHost& h = E->cls[c];
        hipLaunchKernelGGL(k_ens_energy<float>, dim3((unsigned)h.runs.size()), dim3(256), 0, E->stream, d.cls[c],
                           E->eout);
        std::vector<double> part(h.runs.size());
        if (hipMemcpyAsync(part.data(), E->eout, sizeof(double) * h.runs.size(), hipMemcpyDeviceToHost, E->stream) !=
                hipSuccess ||
            hipStreamSynchronize(E->stream) != hipSuccess)
            return efail(E, PST_ERR_HIP, "energy readback failed");
        for (size_t i = 0; i < h.runs.size(); ++i) per_run[h.runs[i]] = part[i];
    }
    for (int r = 0; r < E->nruns; ++r)
        if (!isfinite(per_run[r])) return efail(E, PST_ERR_NONFINITE, "run %d energy is not finite", r);
    return PST_OK;
}

// --------------------------------------------------------------- autotuner
// The persistent kernel's variant is timed on full persistent steps; then, for
// each class in turn (the others fixed at their current choice), the variant
// of its batched launches on full batched steps; then the two graph modes.
// Results are cached in a flat JSON object {"<key>": <variant>,
// "<key>/class<c>": <variant>, "<key>/mode": <mode>} at cache_path (NULL: no
// cache).  The ensemble state is saved and restored around the timing runs.
static std::string arch_name() {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

static std::map<std::string, int> read_cache(const char* path) {
    std::map<std::string, int> m;
    if (!path) return m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t c = s.find(':', j);
        if (c == std::string::npos) break;
        m[key] = atoi(s.c_str() + c + 1);
        i = s.find_first_of(",}", c);
        if (i == std::string::npos) break;
    }
    return m;
}

static void write_cache(const char* path, const std::map<std::string, int>& m) {
    if (!path) return;
    std::ofstream f(path);
    f << "{";
    bool first = true;
    for (auto& kv : m) {
        f << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
        first = false;
    }
    f << "}\n";
}

extern "C" pst_status pst_ensemble_autotune(pst_ensemble* E, const char* cache_path, int force, int* chosen) {
    if (!E) return PST_ERR_INVALID_ARG;
    std::string key = arch_name() + "/ensemble/fp32/rk" + std::to_string(E->p.rk_order) + "/n";
    for (size_t c = 0; c < E->cls.size(); ++c)
        key += (c ? "-" : "") + std::to_string(E->cls[c].n) + "x" + std::to_string(E->cls[c].runs.size());
    std::map<std::string, int> cache = read_cache(cache_path);
    const std::string mkey = key + "/mode";
    auto ckey = [&](size_t c) { return key + "/class" + std::to_string(c); };
    auto valid = [&](const std::string& k) { return cache.count(k) && cache[k] >= 0 && cache[k] < ENS_NVAR; };
    const bool graph_mode = E->mode == 0 || E->mode == 4;
    bool cached = !force && valid(key);
    for (size_t c = 0; cached && c < E->cls.size(); ++c) cached = valid(ckey(c));
    if (cached) {
        drop_graph(E);
        E->var = cache[key];
        for (size_t c = 0; c < E->cls.size(); ++c) E->cvar[c] = cache[ckey(c)];
        if (graph_mode && cache.count(mkey) && (cache[mkey] == 0 || cache[mkey] == 4)) E->mode = cache[mkey];
        if (chosen) *chosen = E->var;
        return PST_OK;
    }
    const int saved_mode = E->mode;
    // save the state: the timing steps overwrite it
    std::vector<std::vector<char>> saved(E->cls.size());
    for (size_t c = 0; c < E->cls.size(); ++c) {
        const size_t b = E->cls[c].runs.size() * 3 * E->cls[c].geo.sc * 8;
        saved[c].resize(b);
        if (hipMemcpy(saved[c].data(), E->cls[c].U, b, hipMemcpyDeviceToHost) != hipSuccess)
            return efail(E, PST_ERR_HIP, "saving state failed");
    }
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    // milliseconds of 3 steps in the current mode, variant and class variants
    auto time_steps = [&](float& ms) -> pst_status {
        launch_step(E);  // warm-up
        hipEventRecord(a, E->stream);
        for (int it = 0; it < 3; ++it) launch_step(E);
        hipEventRecord(b, E->stream);
        if (hipEventSynchronize(b) != hipSuccess) return efail(E, PST_ERR_HIP, "autotune timing failed");
        hipEventElapsedTime(&ms, a, b);
        return E->mode <= 1 ? check_err_flag(E) : PST_OK;
    };
    pst_status st = PST_OK;
    // 1. the persistent kernel's variant (one for all classes: one kernel)
    E->mode = 1;
    drop_graph(E);
    float best = 1e30f;
    int bestv = E->var;
    for (int v = 0; v < ENS_NVAR && st == PST_OK; ++v) {
        E->var = v;
        float ms = 0.f;
        st = time_steps(ms);
        if (st == PST_OK && ms < best) {
            best = ms;
            bestv = v;
        }
    }
    E->var = bestv;
    // 2. each class's variant for the batched launches, the other classes
    // fixed at their current choice (starting from the persistent pick)
    E->mode = 2;
    for (size_t c = 0; c < E->cls.size(); ++c) E->cvar[c] = bestv;
    for (size_t c = 0; c < E->cls.size() && st == PST_OK; ++c) {
        float cbest = 1e30f;
        int cv = E->cvar[c];
        for (int v = 0; v < ENS_NVAR && st == PST_OK; ++v) {
            E->cvar[c] = v;
            float ms = 0.f;
            st = time_steps(ms);
            if (st == PST_OK && ms < cbest) {
                cbest = ms;
                cv = v;
            }
        }
        E->cvar[c] = cv;
    }
    // 3. the graph modes: one persistent launch per step against the batched
    // launches, each replayed from its graph
    int mode_pick = saved_mode;
    if (st == PST_OK && graph_mode) {
        float tbest = 1e30f;
        for (int m : {0, 4}) {
            E->mode = m;
            drop_graph(E);
            st = pst_ensemble_step(E, 1);  // captures the graph, warms up
            if (st != PST_OK) break;
            hipEventRecord(a, E->stream);
            for (int it = 0; it < 3; ++it) hipGraphLaunch(E->gexec, E->stream);
            hipEventRecord(b, E->stream);
            if (hipEventSynchronize(b) != hipSuccess) {
                st = efail(E, PST_ERR_HIP, "autotune timing failed");
                break;
            }
            float ms = 0.f;
            hipEventElapsedTime(&ms, a, b);
            if (m == 0) st = check_err_flag(E);
            if (st == PST_OK && ms < tbest) {
                tbest = ms;
                mode_pick = m;
            }
        }
        drop_graph(E);
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    for (size_t c = 0; c < E->cls.size(); ++c)
        hipMemcpy(E->cls[c].U, saved[c].data(), saved[c].size(), hipMemcpyHostToDevice);
    E->mode = mode_pick;
    if (st != PST_OK) return st;
    cache[key] = bestv;
    for (size_t c = 0; c < E->cls.size(); ++c) cache[ckey(c)] = E->cvar[c];
    if (graph_mode) cache[mkey] = mode_pick;
    write_cache(cache_path, cache);
    if (chosen) *chosen = bestv;
    return PST_OK;
}

extern "C" pst_status pst_ensemble_set_schedule(pst_ensemble* E, int variant) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (variant < 0 || variant >= ENS_NVAR) return efail(E, PST_ERR_INVALID_ARG, "variant %d", variant);
    drop_graph(E);
    E->var = variant;
    for (int c = 0; c < ENS_MAX_CLASSES; ++c) E->cvar[c] = variant;
    return PST_OK;
}

extern "C" pst_status pst_ensemble_set_class_schedule(pst_ensemble* E, int cls, int variant) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (cls < 0 || cls >= (int)E->cls.size()) return efail(E, PST_ERR_INVALID_ARG, "class %d", cls);
    if (variant < 0 || variant >= ENS_NVAR) return efail(E, PST_ERR_INVALID_ARG, "variant %d", variant);
    drop_graph(E);
    E->cvar[cls] = variant;
    return PST_OK;
}

extern "C" pst_status pst_ensemble_class_schedules(const pst_ensemble* E, int* variants) {
    if (!E || !variants) return PST_ERR_INVALID_ARG;
    for (size_t c = 0; c < E->cls.size(); ++c) variants[c] = E->cvar[c];
    return PST_OK;
}

extern "C" pst_status pst_ensemble_query(const pst_ensemble* E, int* nclasses, int* class_n, int* class_runs,
                                         int* variant, int* grid) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (nclasses) *nclasses = (int)E->cls.size();
    for (size_t c = 0; c < E->cls.size(); ++c) {
        if (class_n) class_n[c] = E->cls[c].n;
        if (class_runs) class_runs[c] = (int)E->cls[c].runs.size();
    }
    if (variant) *variant = E->var;
    if (grid) *grid = E->grids[E->var];
    return PST_OK;
}

extern "C" pst_status pst_ensemble_project(pst_ensemble* E) {
    if (!E) return PST_ERR_INVALID_ARG;
    EnsDesc<float> d = make_desc(E, false);
    for (int c = 0; c < d.ncls; ++c)
        hipLaunchKernelGGL(k_ens_project<float>, dim3(512), dim3(256), 0, E->stream, d.cls[c]);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PST_OK : efail(E, PST_ERR_HIP, "projection launch failed");
}

extern "C" pst_status pst_ensemble_diagnostics(pst_ensemble* E, double* energy, double* enstrophy) {
    if (!E) return PST_ERR_INVALID_ARG;
    if (!energy || !enstrophy) return efail(E, PST_ERR_INVALID_ARG, "NULL output");
    EnsDesc<float> d = make_desc(E, false);
    for (int c = 0; c < d.ncls; ++c) {
        const EnsClassHost& h = E->cls[c];
        const size_t R = h.runs.size();
        hipLaunchKernelGGL(k_ens_diag<float>, dim3((unsigned)R), dim3(256), 0, E->stream, d.cls[c], E->eout,
                           E->eout + R);
        std::vector<double> part(2 * R);
        if (hipMemcpyAsync(part.data(), E->eout, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, E->stream) !=
                hipSuccess ||
            hipStreamSynchronize(E->stream) != hipSuccess)
            return efail(E, PST_ERR_HIP, "diagnostics readback failed");
        for (size_t i = 0; i < R; ++i) {
            energy[h.runs[i]] = part[i];
            enstrophy[h.runs[i]] = part[R + i];
        }
    }
    for (int r = 0; r < E->nruns; ++r)
        if (!isfinite(energy[r]) || !isfinite(enstrophy[r])) return efail(E, PST_ERR_NONFINITE, "run %d diagnostics", r);
    return PST_OK;
}

extern "C" pst_status pst_ensemble_rel_l2(pst_ensemble* A, const pst_ensemble* Bn, double* per_run) {
    if (!A || !Bn) return PST_ERR_INVALID_ARG;
    if (!per_run) return efail(A, PST_ERR_INVALID_ARG, "NULL output");
    if (A->nruns != Bn->nruns || A->cls.size() != Bn->cls.size()) return efail(A, PST_ERR_INVALID_ARG, "ensembles differ");
    for (size_t c = 0; c < A->cls.size(); ++c)
        if (A->cls[c].n != Bn->cls[c].n || A->cls[c].runs != Bn->cls[c].runs)
            return efail(A, PST_ERR_INVALID_ARG, "ensembles differ");
    EnsDesc<float> da = make_desc(A, false), db = make_desc(const_cast<pst_ensemble*>(Bn), false);
    for (int c = 0; c < da.ncls; ++c) {
        const EnsClassHost& h = A->cls[c];
        const size_t R = h.runs.size();
        hipLaunchKernelGGL(k_ens_dist<float>, dim3((unsigned)R), dim3(256), 0, A->stream, da.cls[c], db.cls[c], A->eout);
        std::vector<double> part(2 * R);
        if (hipMemcpyAsync(part.data(), A->eout, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, A->stream) !=
                hipSuccess ||
            hipStreamSynchronize(A->stream) != hipSuccess)
            return efail(A, PST_ERR_HIP, "readback failed");
        for (size_t i = 0; i < R; ++i) per_run[h.runs[i]] = sqrt(part[2 * i] / part[2 * i + 1]);
    }
    return PST_OK;
}
