// Device side of the ensemble path (see ensemble.hip): schedules, per-unit
// dispatch over the grid sizes of an ensemble, the persistent step kernel
// with its bounded device-wide barrier, and the per-pass kernels.
#pragma once
#include <algorithm>

#include "kernels.h"

namespace pst {

constexpr int ENS_NT = 256;          // threads per block of the ensemble kernels
constexpr int ENS_MAX_CLASSES = 4;
constexpr int ENS_NVAR = 4;          // schedules: 2 radix orders x 2 tile sizes

// --------------------------------------------------------------- schedules
// Radix orders per n (every thread holds E = n / G points; E <= 12 keeps the
// persistent kernel's register footprint modest).
template <int N, int PV> struct EnsPlan;
template <> struct EnsPlan<32, 0> { using P = Radices<8, 4>; static constexpr int G = 4; };
template <> struct EnsPlan<32, 1> { using P = Radices<4, 8>; static constexpr int G = 4; };
template <> struct EnsPlan<48, 0> { using P = Radices<4, 4, 3>; static constexpr int G = 4; };
template <> struct EnsPlan<48, 1> { using P = Radices<3, 4, 4>; static constexpr int G = 4; };
template <> struct EnsPlan<64, 0> { using P = Radices<8, 8>; static constexpr int G = 8; };
template <> struct EnsPlan<64, 1> { using P = Radices<4, 4, 4>; static constexpr int G = 16; };
template <> struct EnsPlan<96, 0> { using P = Radices<4, 4, 3, 2>; static constexpr int G = 8; };
template <> struct EnsPlan<96, 1> { using P = Radices<2, 4, 4, 3>; static constexpr int G = 8; };

// variant v: radix order v & 1, tile lines (v & 2) ? TL/2 : TL
template <typename T, int N, int V>
using EnsCfg = KCfg<typename EnsPlan<N, V & 1>::P, EnsPlan<N, V & 1>::G, (V & 2) ? tile_lines<T>() / 2 : tile_lines<T>()>;
template <typename T, int N, int V>
using EnsLineCfg = KCfg<typename EnsPlan<N, V & 1>::P, EnsPlan<N, V & 1>::G, 1>;

inline bool ens_supported_n(int n) { return n == 32 || n == 48 || n == 64 || n == 96; }

template <typename T>
struct EnsClass {
    Geo geo;
    int nruns;
    cx<T>*U, *V, *Acc, *A, *B, *C;
    int64_t s_st, s_a, s_b, s_c;  // per-run strides (elements)
    const cx<T>* tw;
    const T* E;
    const T* E2;
    int64_t upr[5];               // work units per run for each pass
};

template <typename T>
struct EnsDesc {
    int ncls;
    EnsClass<T> cls[ENS_MAX_CLASSES];
    int nstages;
    int modes[4];
    T h;
    unsigned* bar;
    int* err;
    long long spin_limit;
};

// LDS elements of the largest body over all classes / variants
template <typename T>
constexpr int ens_lds() {
    int m = 0;
    // line bodies: (NT / G) lines of n + n/8
    const int lines[][2] = {{32, 4}, {48, 4}, {64, 8}, {64, 16}, {96, 8}};
    for (auto& l : lines) m = std::max(m, (ENS_NT / l[1]) * (l[0] + l[0] / 8));
    const int tiles[][2] = {{32, 4}, {48, 4}, {64, 8}, {64, 16}, {96, 8}};
    for (auto& t : tiles)
        for (int tl : {tile_lines<T>(), tile_lines<T>() / 2})
            if (t[1] * tl <= ENS_NT) m = std::max(m, (ENS_NT / (t[1] * tl)) * t[0] * (tl + 1));
    return m;
}

// units per run of each pass for class geometry g and variant var
template <typename T, int N, int V>
inline void ens_units_v(const Geo& g, int64_t* upr) {
    using TC = EnsCfg<T, N, V>;
    using LC = EnsLineCfg<T, N, V>;
    upr[0] = line_units<LC, ENS_NT>(g);
    upr[1] = ytile_units<TC, ENS_NT>(g, 6);
    upr[2] = xtile_units<TC, ENS_NT>(g);
    upr[3] = ytile_units<TC, ENS_NT>(g, 3);
    upr[4] = line_units<LC, ENS_NT>(g);
}
template <typename T, int V>
inline void ens_units(const Geo& g, int64_t* upr) {
    switch (g.n) {
        case 32: ens_units_v<T, 32, V>(g, upr); break;
        case 48: ens_units_v<T, 48, V>(g, upr); break;
        case 64: ens_units_v<T, 64, V>(g, upr); break;
        default: ens_units_v<T, 96, V>(g, upr); break;
    }
}

// One work unit of one pass of one run.
template <typename T, int N, int V>
__device__ __forceinline__ void ens_unit_v(const EnsClass<T>& c, int pass, int stage_in_v, int mode, T h, int run,
                                           int64_t lu, cx<T>* sm) {
    using TC = EnsCfg<T, N, V>;
    using LC = EnsLineCfg<T, N, V>;
    const Geo& g = c.geo;
    const int tid = threadIdx.x;
    cx<T>* A = c.A + run * c.s_a;
    cx<T>* B = c.B + run * c.s_b;
    cx<T>* C = c.C + run * c.s_c;
    switch (pass) {
        case 0: {
            const cx<T>* st = (stage_in_v ? c.V : c.U) + run * c.s_st;
            zinv_body<T, LC, ENS_NT, 1>(st, A, c.tw, g, lu, tid, sm);
        } break;
        case 1: ypass_body<T, TC, ENS_NT, true, TC::N>(A, B, c.tw, g, g.sa, g.sb, 6, lu, tid, sm); break;
        // ensemble grids use the 2/3 rule: the cutoff is compiled in
        case 2: xpass_body<T, TC, ENS_NT, 0, false, false, (N + 2) / 3 - 1>(B, C, c.tw, g, lu, tid, sm); break;
        case 3: ypass_body<T, TC, ENS_NT, false, TC::N>(C, A, c.tw, g, g.sb, g.sa, 3, lu, tid, sm); break;
        default: {
            RkArgs<T> ra;
            ra.U = c.U + run * c.s_st;
            ra.V = c.V + run * c.s_st;
            ra.Acc = c.Acc + run * c.s_st;
            ra.R = nullptr;
            ra.E[0] = ra.E[1] = c.E;
            ra.E2[0] = ra.E2[1] = c.E2;
            ra.h = h;
            ra.F = nullptr;
            ra.kf = -1;
            ra.lin_only = 0;
            ra.sph2 = -1;
            zfwd_body<T, LC, ENS_NT, 0>(A, c.tw, g, ra, mode, lu, tid, sm);
        } break;
    }
}

template <typename T, int V>
__device__ __forceinline__ void ens_unit(const EnsClass<T>& c, int pass, int sv, int mode, T h, int run, int64_t lu,
                                         cx<T>* sm) {
    switch (c.geo.n) {
        case 32: ens_unit_v<T, 32, V>(c, pass, sv, mode, h, run, lu, sm); break;
        case 48: ens_unit_v<T, 48, V>(c, pass, sv, mode, h, run, lu, sm); break;
        case 64: ens_unit_v<T, 64, V>(c, pass, sv, mode, h, run, lu, sm); break;
        default: ens_unit_v<T, 96, V>(c, pass, sv, mode, h, run, lu, sm); break;
    }
}

// Device-wide barrier with a bounded wait.  Returns false (on every thread of
// the block) if the barrier failed or another block reported a failure.
// Arrivals are counted in ENS_BAR_SUB sub-counters (block b in group
// b % ENS_BAR_SUB), each on its own cache line, so that no single atomic
// location serialises every block; the last arrival of a group then counts the
// group in, and the last group releases a new generation, which the waiting
// blocks poll with relaxed loads.  One agent-scope release fence per block
// before it arrives and one acquire fence after it leaves (each writes back /
// invalidates non-coherent caches, so none sits in the polling loop); group
// and final leaders acquire what they count in and release it onwards.
//   bar[0]: groups arrived; bar[32]: generation; bar[64 + 32 g]: group g
constexpr int ENS_BAR_SUB = 16;
constexpr int ENS_BAR_WORDS = 32 * (2 + ENS_BAR_SUB);
__device__ __forceinline__ bool grid_barrier(unsigned* bar, int* err, unsigned nblocks, long long limit) {
    __shared__ int ok_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned gen = __hip_atomic_load(&bar[32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned g = blockIdx.x % ENS_BAR_SUB;
        const unsigned ngroups = nblocks < (unsigned)ENS_BAR_SUB ? nblocks : (unsigned)ENS_BAR_SUB;
        const unsigned gsize = (nblocks - g + ENS_BAR_SUB - 1) / ENS_BAR_SUB;
        unsigned* sub = &bar[64 + 32 * g];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned a = __hip_atomic_fetch_add(sub, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == gsize - 1) {
            __hip_atomic_store(sub, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const unsigned t = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ngroups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(&bar[32], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        long long spins = 0;
        while (__hip_atomic_load(&bar[32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
            if (++spins > limit) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok_sh = ok;
    }
    __syncthreads();
    return ok_sh != 0;
}

// The units of one pass of one class, handed out round-robin over the grid;
// `first` is the global index of the class's first unit (units of all
// classes of a pass form one sequence, largest grids first).
template <typename T, int N, int V>
__device__ __forceinline__ void ens_class_pass(const EnsClass<T>& c, int pass, int sv, int mode, T h, int64_t first,
                                               cx<T>* sm) {
    const int64_t upr = c.upr[pass], total = c.nruns * upr;
    int64_t u = ((int64_t)blockIdx.x - first) % gridDim.x;
    if (u < 0) u += gridDim.x;
    for (; u < total; u += gridDim.x) ens_unit_v<T, N, V>(c, pass, sv, mode, h, (int)(u / upr), u % upr, sm);
}

template <typename T, int V>
__global__ __launch_bounds__(ENS_NT, 2) void k_ens_persistent(const EnsDesc<T>* __restrict__ dp) {
    __shared__ cx<T> sm[ens_lds<T>()];
    const EnsDesc<T>& d = *dp;   // device-resident descriptor
    if (__hip_atomic_load(d.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    for (int s = 0; s < d.nstages; ++s) {
        for (int pass = 0; pass < 5; ++pass) {
            int64_t first = 0;
            for (int c = 0; c < d.ncls; ++c) {
                const EnsClass<T>& cl = d.cls[c];
                switch (cl.geo.n) {
                    case 32: ens_class_pass<T, 32, V>(cl, pass, s > 0, d.modes[s], d.h, first, sm); break;
                    case 48: ens_class_pass<T, 48, V>(cl, pass, s > 0, d.modes[s], d.h, first, sm); break;
                    case 64: ens_class_pass<T, 64, V>(cl, pass, s > 0, d.modes[s], d.h, first, sm); break;
                    default: ens_class_pass<T, 96, V>(cl, pass, s > 0, d.modes[s], d.h, first, sm); break;
                }
                first += cl.nruns * cl.upr[pass];
            }
            if (!grid_barrier(d.bar, d.err, gridDim.x, d.spin_limit)) return;
        }
    }
}

// one pass of one class, all its runs (BATCHED mode); blockIdx.x = unit
template <typename T, int V>
__global__ __launch_bounds__(ENS_NT, 2) void k_ens_pass(EnsClass<T> c, int pass, int sv, int mode, T h) {
    __shared__ cx<T> sm[ens_lds<T>()];
    const int64_t upr = c.upr[pass];
    const int64_t u = blockIdx.x;
    ens_unit<T, V>(c, pass, sv, mode, h, (int)(u / upr), u % upr, sm);
}

// one pass of one run (SEQUENTIAL mode)
template <typename T, int V>
__global__ __launch_bounds__(ENS_NT, 2) void k_ens_pass_run(EnsClass<T> c, int pass, int sv, int mode, T h, int run) {
    __shared__ cx<T> sm[ens_lds<T>()];
    ens_unit<T, V>(c, pass, sv, mode, h, run, blockIdx.x, sm);
}


// Host-callable entry points of one schedule variant (one per translation unit)
struct EnsKernels {
    void (*units)(const Geo&, int64_t*);
    const void* persistent;  // k_ens_persistent<float, V>
    void (*launch_persistent)(const EnsDesc<float>* dev_desc, int grid, hipStream_t);
    void (*launch_pass)(const EnsClass<float>&, int pass, int sv, int mode, float h, hipStream_t);
    void (*launch_pass_run)(const EnsClass<float>&, int pass, int sv, int mode, float h, int run, hipStream_t);
};

template <int V>
struct EnsVariant {
    static void launch_persistent(const EnsDesc<float>* d, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_ens_persistent<float, V>), dim3(grid), dim3(ENS_NT), 0, s, d);
    }
    static void launch_pass(const EnsClass<float>& c, int pass, int sv, int mode, float h, hipStream_t s) {
        hipLaunchKernelGGL((k_ens_pass<float, V>), dim3((unsigned)(c.nruns * c.upr[pass])), dim3(ENS_NT), 0, s, c,
                           pass, sv, mode, h);
    }
    static void launch_pass_run(const EnsClass<float>& c, int pass, int sv, int mode, float h, int run, hipStream_t s) {
        hipLaunchKernelGGL((k_ens_pass_run<float, V>), dim3((unsigned)c.upr[pass]), dim3(ENS_NT), 0, s, c, pass, sv,
                           mode, h, run);
    }
    static const EnsKernels* get() {
        static const EnsKernels k = {&ens_units<float, V>, (const void*)&k_ens_persistent<float, V>, &launch_persistent,
                                     &launch_pass, &launch_pass_run};
        return &k;
    }
};

}  // namespace pst

#define PST_ENS_VARIANT(VV) \
    namespace pst {         \
    const EnsKernels* ens_kernels_v##VV() { return EnsVariant<VV>::get(); } \
    }
