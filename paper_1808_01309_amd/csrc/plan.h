// Internal plan state shared by the runtime and the per-size kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pst.h"

namespace pst {

// Geometry of the dealiased pass buffers.  Each axis has its own point count
// and cutoff (Sec. 2 lets N_x, N_y, N_z and the box lengths differ); the
// fields without a suffix describe the z axis, and for cubic grids all three
// axes are equal.
//   K   dealias cutoff, M = 2K + 1 kept wavenumbers on a full axis (z);
//   Ky, My the same for y; Kx for x, nxk = Kx + 1 kept kx on the half axis.
// Compact index j in [0, M) <-> wavenumber j (j <= K) or j - M (j > K)
//                         <-> FFT position j (j <= K) or j + n - M.
// Buffers (complex, element type of the plan):
//   state   [ncomp][nxk][My][M]   (kx, jy, jz)       component stride sc
//   A, D    [nf][nxk][My][n]      (kx, jy, z)        field stride sa
//   B, C    [nf][nxk][ny][n]      (kx, y, z)         field stride sb, kx plane
//           stride pb = ny n + BC_PAD: the unpadded plane stride is a power
//           of two for the power-of-two grids (2 MB at 512^3 FP32), and the x
//           pass, which reads one short z row from each kx plane, then spreads
//           its reads over few memory channels (a memory-only kernel with the
//           x pass's 512^3 access pattern: 1.03 ms unpadded, 0.72 ms padded)
//   full = 1 (Gross-Pitaevskii): kx runs over the whole axis like ky and kz
//   (compact index jx in [0, 2Kx + 1), nxk = 2Kx + 1); full = 0: kx = jx in [0, Kx].
// Physical wavenumber of index k on axis i: a_i k, a_i = 2 pi / L_i (1 for
// the 2 pi box).  aniso = 0 when all a_i are 1 (|k|^2 is then an integer and
// indexes the integrating-factor tables).
constexpr int BC_PAD = 64;   // elements: keeps 128-byte rows aligned in both precisions
struct Geo {
    int n, K, M, nxk;
    int64_t sc, sa, sb, pb;
    int full;
    int nx, ny, Kx, Ky, My;
    double ax, ay, az;
    int aniso;
};

// Geometry of an nx x ny x nz grid with cutoffs Kx, Ky, Kz, wavenumber scales
// a_i = 2 pi / L_i; full: kx over the whole axis (complex fields).
inline Geo make_geo(int nx, int ny, int nz, int Kx, int Ky, int Kz, double ax, double ay, double az, int full) {
    Geo g{};
    g.n = nz;
    g.K = Kz;
    g.M = 2 * Kz + 1;
    g.nx = nx;
    g.ny = ny;
    g.Kx = Kx;
    g.Ky = Ky;
    g.My = 2 * Ky + 1;
    g.full = full;
    g.nxk = full ? 2 * Kx + 1 : Kx + 1;
    g.sc = (int64_t)g.nxk * g.My * g.M;
    g.sa = (int64_t)g.nxk * g.My * nz;
    g.pb = (int64_t)ny * nz + BC_PAD;
    g.sb = (int64_t)g.nxk * g.pb;
    g.ax = ax;
    g.ay = ay;
    g.az = az;
    g.aniso = (ax != 1.0 || ay != 1.0 || az != 1.0) ? 1 : 0;
    return g;
}

// compact index / FFT position / wavenumber on an axis of n points and cutoff K
__host__ __device__ inline int ax_j_of_pos(int p, int n, int K) { return p <= K ? p : (p >= n - K ? p - (n - 2 * K - 1) : -1); }
__host__ __device__ inline int ax_k_of_j(int j, int K) { return j <= K ? j : j - (2 * K + 1); }
// z axis
__host__ __device__ inline int pos_of_j(int j, const Geo& g) { return j <= g.K ? j : j + g.n - g.M; }
__host__ __device__ inline int j_of_pos(int p, const Geo& g) {
    return p <= g.K ? p : (p >= g.n - g.K ? p - (g.n - g.M) : -1);
}
__host__ __device__ inline int k_of_j(int j, const Geo& g) { return j <= g.K ? j : j - g.M; }
// y axis
__host__ __device__ inline int jy_of_pos(int p, const Geo& g) { return ax_j_of_pos(p, g.ny, g.Ky); }
__host__ __device__ inline int ky_of_j(int j, const Geo& g) { return ax_k_of_j(j, g.Ky); }
// x axis (full axes only: the half axis has kx = jx)
__host__ __device__ inline int jx_of_pos(int p, const Geo& g) { return ax_j_of_pos(p, g.nx, g.Kx); }
__host__ __device__ inline int kx_of_j(int j, const Geo& g) { return g.full ? ax_k_of_j(j, g.Kx) : j; }
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
    const pst::Launchers* L;   // z axis (all axes of a cubic grid; the neural operator's transforms)
    const pst::Launchers *Lx, *Ly;
    // device buffers
    void *U, *V, *Acc;       // state, stage input, RK accumulator (compact)
    void *A, *B, *C;         // pass buffers (D aliases A)
    void *tw;                // nz roots of unity
    void *twy, *twx;         // ny / nx roots (alias tw or each other where the lengths agree)
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
    // one axis of the standalone transforms (composed by the runtime):
    // contiguous x lines (real <-> half spectrum, or complex), and complex
    // transforms down strided columns (y, z)
    void (*fftx_r2c)(pst_plan*, const void* in, void* out, int64_t nlines);
    void (*fftx_c2r)(pst_plan*, const void* in, void* out, int64_t nlines);
    void (*fftx_c2c)(pst_plan*, const void* in, void* out, int64_t nlines, int inverse);
    void (*fft_cols)(pst_plan*, const void* in, void* out, int64_t rs, int64_t ncols, int64_t ps, int64_t nplanes,
                     int inverse, double scale, int kind);
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
