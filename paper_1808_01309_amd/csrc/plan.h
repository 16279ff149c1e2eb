// Internal plan state shared by the runtime and the per-size kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pst.h"

namespace pst {

// Geometry of the dealiased pass buffers.
//   K   dealias cutoff, M = 2K + 1 kept wavenumbers on a full axis,
//   nxk = K + 1 kept wavenumbers on the half x axis.
// Compact index j in [0, M) <-> wavenumber j (j <= K) or j - M (j > K)
//                         <-> FFT position j (j <= K) or j + n - M.
// Buffers (complex, element type of the plan):
//   state   [ncomp][nxk][M][M]   (kx, jy, jz)       component stride sc
//   A, D    [nf][nxk][M][n]      (kx, jy, z)        field stride sa
//   B, C    [nf][nxk][n][n]      (kx, y, z)         field stride sb
//   full = 1 (Gross-Pitaevskii): kx runs over the whole axis like ky and kz
//   (compact index jx in [0, M), nxk = M); full = 0: kx = jx in [0, K].
struct Geo {
    int n, K, M, nxk;
    int64_t sc, sa, sb;
    int full;
};

__host__ __device__ inline int pos_of_j(int j, const Geo& g) { return j <= g.K ? j : j + g.n - g.M; }
__host__ __device__ inline int j_of_pos(int p, const Geo& g) {
    return p <= g.K ? p : (p >= g.n - g.K ? p - (g.n - g.M) : -1);
}
__host__ __device__ inline int k_of_j(int j, const Geo& g) { return j <= g.K ? j : j - g.M; }
__host__ __device__ inline int k_of_pos(int p, int n) { return p < n / 2 ? p : p - n; }

// RK stage selector of the forward z pass
enum ZMode {
    Z_RHS = 0,                                  // write N(u) to rhs buffer
    Z_RK4_0 = 1, Z_RK4_1 = 2, Z_RK4_2 = 3, Z_RK4_3 = 4,
    Z_RK2_0 = 5, Z_RK2_1 = 6
};

struct Launchers;

}  // namespace pst

struct TimerRec {
    int kind;
    hipEvent_t a, b;
};

struct pst_plan {
    pst_params p;
    hipStream_t stream;
    pst::Geo geo;
    int ncomp, nfin, nfout;  // state components, backward fields, forward fields
    size_t esz;              // bytes per complex element
    const pst::Launchers* L;
    // device buffers
    void *U, *V, *Acc;       // state, stage input, RK accumulator (compact)
    void *A, *B, *C;         // pass buffers (D aliases A)
    void *tw;                // n roots of unity
    void *Etab[2], *E2tab[2];  // integrating factors by |k|^2 for u and b
    void *force;             // forcing box [3][kf+1][2kf+1][2kf+1] or null
    int kf;
    void *abi;               // spectral scratch in the ABI layout (lazily allocated)
    size_t abi_bytes;
    double* red;             // reduction partials + results
    size_t owned_bytes;
    long long steps;
    std::string err;
    // timers
    std::vector<TimerRec> pending;
    std::vector<hipEvent_t> pool;
    double t_ms[PST_K_COUNT];
    long long t_cnt[PST_K_COUNT];
};

namespace pst {

// Scoped timer around kernel launches of one kind.
struct KTimer {
    pst_plan* P;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(pst_plan* plan, int k);
    ~KTimer();
};

// Per-(n, precision) kernel launchers.
struct Launchers {
    int n;
    int radices[4];
    int tile_lines;
    void (*zinv)(pst_plan*, const void* state);
    void (*yinv)(pst_plan*);
    void (*xpass)(pst_plan*);
    void (*yfwd)(pst_plan*);
    void (*zfwd)(pst_plan*, int mode, void* rhs_out);
    void (*fft_r2c)(pst_plan*, const void* in, void* out, int nf);
    void (*fft_c2r)(pst_plan*, const void* in, void* out, int nf, void* tmp);
    // complex 3D transform [nf][n][n][n] (x fastest), forward (sign -, 1/n^3) or
    // inverse (sign +, unscaled); in == out allowed
    void (*fft_c2c)(pst_plan*, const void* in, void* out, int nf, int inverse);
    // transforms restricted to the retained-mode box (kx < m, ky, kz in [0, m) U [n-m, n)),
    // compact spectra [nf][2m][2m][m]; workspace nf n n m + nf n 2m m complex
    void (*fft_r2c_modes)(pst_plan*, const void* in, void* out, int nf, int m, void* tmp);
    void (*fft_c2r_modes)(pst_plan*, const void* in, void* out, int nf, int m, void* tmp);
    // their y and z passes alone: from / to the x-transformed lines held in the
    // first nf n n m complex of the workspace
    void (*modes_yz_fwd)(pst_plan*, void* out, int nf, int m, void* tmp);
    void (*modes_yz_inv)(pst_plan*, const void* in, int nf, int m, void* tmp);
};

const Launchers* launchers_for(int n, int precision);

}  // namespace pst
