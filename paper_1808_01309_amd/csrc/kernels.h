// Pass kernels of the pseudospectral right-hand side and of the standalone
// 3D transforms, templated on element type T and grid size N.
//
// Right-hand side (Sec. 2: products in physical space, projection in
// spectral space; transform steps as in the slab algorithm of Sec. 2 with the
// global transpose replaced by on-device strided passes):
//   zinv   state (kept modes)  -> curl in registers -> backward z  -> A
//   yinv   A (kept ky rows)    -> backward y                       -> B
//   xpass  B (kx <= K rows)    -> backward x (c2r), u x w (+ j x b, u x b),
//                                 forward x (r2c), keep kx <= K    -> C
//   yfwd   C                   -> forward y, keep kept ky rows     -> D (= A)
//   zfwd   D                   -> forward z, keep kept kz, 1/n^3, projection
//                                 (or curl for b), forcing, RK stage update
// Only modes inside the dealiasing cube are ever read or written, so the
// transforms are pruned on both ends; physical-space fields never touch HBM.
#pragma once
#include <type_traits>

#include "fft_engine.h"
#include "plan.h"

namespace pst {

// ------------------------------------------------------------ size configs
// Radix schedule and threads per line for every supported n.
template <int N> struct NCfg;
template <> struct NCfg<16>   { using P = Radices<4, 4>;    static constexpr int G = 4; };
template <> struct NCfg<24>   { using P = Radices<4, 2, 3>; static constexpr int G = 2; };
template <> struct NCfg<32>   { using P = Radices<8, 4>;    static constexpr int G = 4; };
template <> struct NCfg<48>   { using P = Radices<4, 4, 3>; static constexpr int G = 4; };
template <> struct NCfg<64>   { using P = Radices<8, 8>;    static constexpr int G = 8; };
template <> struct NCfg<96>   { using P = Radices<8, 4, 3>; static constexpr int G = 4; };
template <> struct NCfg<128>  { using P = Radices<4, 8, 4>; static constexpr int G = 16; };
template <> struct NCfg<256>  { using P = Radices<4, 8, 8>; static constexpr int G = 32; };
template <> struct NCfg<512>  { using P = Radices<8, 8, 8>; static constexpr int G = 64; };
template <> struct NCfg<1024> { using P = Radices<8, 16, 8>; static constexpr int G = 64; };

// Lines per workgroup of the strided passes: 128-byte row segments.
template <typename T> constexpr int tile_lines() { return sizeof(T) == 4 ? 16 : 8; }
// The x pass keeps every field of a line in registers until the products are
// formed: MHD (twice the fields) and n = 1024 (twice the points per thread)
// each halve the tile so the block stays within the register file.
template <typename T, bool MHD, int N>
constexpr int xpass_lines() {
    // FP32 Navier-Stokes: 8 lines below n = 1024, 4 at 1024 (128 threads per
    // line there), two workgroups per CU
    if (sizeof(T) == 4 && !MHD) return N < 1024 ? 8 : 4;
    // FP32 MHD at n = 1024: 4 lines of 128 threads (172 VGPRs, one 512-thread
    // workgroup per CU), whose 32-byte rows of the padded kx planes read
    // faster than the 16-byte rows of 2-line tiles (x pass 41.1 -> 32.8 ms at
    // 1024^3; halving the 512^3 Boussinesq tile measured 2.95 -> 4.62 ms)
    if (sizeof(T) == 4 && N >= 1024) return 4;
    return tile_lines<T>() / (MHD ? 2 : 1) / (N >= 1024 ? 2 : 1);
}
constexpr int LINE_BLOCK = 256;

// A kernel configuration: radix schedule P (length N), G threads per line,
// TL lines per tile of the strided passes.
template <class P_, int G_, int TL_>
struct KCfg {
    using P = P_;
    static constexpr int N = P_::N, G = G_, TL = TL_;
};
// z passes (one line per G threads): at n = 1024 a line is spread over 128
// threads (8 points each, radices 8 8 4 4) so that the curl / projection / RK
// bodies stay within a register budget that lets several wavefronts share a SIMD.
template <int N> struct LPlan {
    using P = typename NCfg<N>::P;
    static constexpr int G = NCfg<N>::G;
};
template <> struct LPlan<1024> {
    using P = Radices<8, 8, 4, 4>;
    static constexpr int G = 128;
};
template <typename T, int N> using LineCfg = KCfg<typename LPlan<N>::P, LPlan<N>::G, 1>;
template <typename T, int N> using TileCfg = KCfg<typename NCfg<N>::P, NCfg<N>::G, tile_lines<T>()>;
// The x pass holds every field of its lines in registers until the products
// are formed; for MHD at n = 1024 (12 fields) it spreads a line over 128
// threads (8 points each, radices 8 8 4 4) so that more wavefronts fit on a
// CU (measured 11% faster than 64 threads x 16 points).
template <typename T, int N, bool MHD> struct XPlan {
    using P = typename NCfg<N>::P;
    static constexpr int G = NCfg<N>::G;
};
template <> struct XPlan<float, 1024, true> {
    using P = Radices<8, 8, 4, 4>;
    static constexpr int G = 128;
};
// Navier-Stokes at n = 1024 likewise: 8 points per thread keep the three
// pairs of a line in about the registers of the 512-point pass
template <> struct XPlan<float, 1024, false> {
    using P = Radices<8, 8, 4, 4>;
    static constexpr int G = 128;
};
template <typename T, int N, bool MHD>
using XCfg = KCfg<typename XPlan<T, N, MHD>::P, XPlan<T, N, MHD>::G, xpass_lines<T, MHD, N>()>;

// LDS elements a body needs for a block of NT threads.
template <typename T, class CF, int NT> constexpr int line_lds() { return (NT / CF::G) * LineLds<T>::size(CF::N); }
template <typename T, class CF, int NT> constexpr int tile_lds() { return (NT / (CF::G * CF::TL)) * CF::N * (CF::TL + 1); }
template <int N, int TL> constexpr int ztiles() { return (N + TL - 1) / TL; }
// z tiles of a plan's z axis (the strided passes transform y or x)
template <int TL> __host__ __device__ inline int zt_count(const Geo& g) { return (g.n + TL - 1) / TL; }

// Workgroups are dispatched to the 8 XCDs round-robin; xcd_unit renumbers
// them so that each XCD works through one contiguous range of units (a
// bijection on [0, gridDim.x)).
__device__ __forceinline__ int64_t xcd_unit() {
    const int64_t nb = gridDim.x, b = blockIdx.x, x = b % 8, q = nb / 8, r = nb % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Work units: a line body handles NT / G lines per unit, a tile body
// NT / (G TL) tiles per unit.
template <class CF, int NT> inline int64_t line_units(const Geo& g) {
    return ((int64_t)g.nxk * g.My + NT / CF::G - 1) / (NT / CF::G);
}
template <class CF, int NT> inline int64_t ytile_units(const Geo& g, int nf) {
    constexpr int SG = NT / (CF::G * CF::TL);
    return ((int64_t)nf * g.nxk * zt_count<CF::TL>(g) + SG - 1) / SG;
}
template <class CF, int NT> inline int64_t xtile_units(const Geo& g) {
    constexpr int SG = NT / (CF::G * CF::TL);
    return ((int64_t)g.ny * zt_count<CF::TL>(g) + SG - 1) / SG;
}

template <typename T>
struct RkArgs {
    cx<T>* U;          // u_n (compact)
    cx<T>* V;          // next stage input
    cx<T>* Acc;        // accumulator
    cx<T>* R;          // rhs output (Z_RHS)
    const T* E[2];     // exp(-visc |k|^2 h / 2) by |k|^2, for u and b
    const T* E2[2];    // exp(-visc |k|^2 h)
    T h;
    const cx<T>* F;    // forcing box or null
    int kf;
    int lin_only;
    int sph2;          // spherical truncation: nonlinear terms kept for |k|^2 <= sph2; -1: the cube
    // Gross-Pitaevskii: unitary factors exp(-i alpha |k|^2 h / 2), exp(-i alpha |k|^2 h)
    // by |k|^2, and the coupling beta of the cubic term
    const cx<T>* Ec;
    const cx<T>* E2c;
    T beta;
    // non-cubic grids (|k|^2 not an integer): the factors are evaluated per
    // mode in FP64 from these (nu or eta / kappa; GPE: alpha in visc[0])
    double visc[2];
    double hd;
};

// ------------------------------------------------------------ zinv + curl
// One line (kx, jy) per G threads.  NGRP = 1 (u) or 2 (u, b): each group of
// 3 state components yields 6 fields: v and i k x v.  THETA (Boussinesq): the
// scalar (state component 3) then yields 4 more fields, i k theta (the
// gradient) and theta itself.
template <typename T, class CF, int NT, int NGRP, bool THETA = false>
__device__ __forceinline__ void zinv_body(const cx<T>* __restrict__ st, cx<T>* __restrict__ A,
                                          const cx<T>* __restrict__ tw, const Geo& geo, int64_t unit, int tid,
                                          cx<T>* sm) {
    constexpr int N = CF::N, G = CF::G;
    // A line's G threads are lanes of one wavefront: the FP64 transforms
    // synchronise per wavefront (measured faster there; FP32 keeps the
    // workgroup barrier, which measured slightly faster for it).
    using F = Fft<T, typename CF::P, G, true, false, sizeof(T) == 8 && G <= 64, sizeof(T) == 4>;
    constexpr int E = F::E, LPB = NT / G, LS = LineLds<T>::size(N);
    const int l = tid / G, g = tid % G;
    const int64_t line = unit * LPB + l;
    const bool active = line < (int64_t)geo.nxk * geo.My;
    const int kx = active ? (int)(line / geo.My) : 0;
    const int jy = active ? (int)(line % geo.My) : 0;
    // physical wavenumbers a_i k_i
    const T fkx = T(geo.ax) * T(kx), fky = T(geo.ay) * T(ky_of_j(jy, geo)), az = T(geo.az);
    const LineLds<T> lds{sm + l * LS};
    const int64_t lin = (int64_t)kx * geo.My + jy;
    for (int grp = 0; grp < NGRP; ++grp) {
        const cx<T>* src = st + (int64_t)(grp * 3) * geo.sc + lin * geo.M;
        cx<T> u[3][E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = j_of_pos(F::first_pos(g, e), geo);
#pragma unroll
            for (int c = 0; c < 3; ++c) u[c][e] = (active && j >= 0) ? src[c * geo.sc + j] : czero<T>();
        }
        // the curl components one at a time (i k x v)_c, then v itself: at
        // most 4 lines live in registers and the state is read once
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<T> w[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T fkz = az * T(k_of_pos(F::first_pos(g, e), N));
                const cx<T> a = u[0][e], b = u[1][e], d = u[2][e];
                if (c == 0) w[e] = mul_i(cx<T>{fky * d.x - fkz * b.x, fky * d.y - fkz * b.y});
                else if (c == 1) w[e] = mul_i(cx<T>{fkz * a.x - fkx * d.x, fkz * a.y - fkx * d.y});
                else w[e] = mul_i(cx<T>{fkx * b.x - fky * a.x, fkx * b.y - fky * a.y});
            }
            F::run(w, g, lds, tw);
            if (active) {
                cx<T>* dst = A + (int64_t)(grp * 6 + 3 + c) * geo.sa + lin * N;
#pragma unroll
                for (int e = 0; e < E; ++e) dst[F::last_pos(g, e)] = w[e];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            F::run(u[c], g, lds, tw);
            if (active) {
                cx<T>* dst = A + (int64_t)(grp * 6 + c) * geo.sa + lin * N;
#pragma unroll
                for (int e = 0; e < E; ++e) dst[F::last_pos(g, e)] = u[c][e];
            }
        }
    }
    if constexpr (THETA) {
        const cx<T>* src = st + (int64_t)3 * geo.sc + lin * geo.M;
        cx<T> th[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = j_of_pos(F::first_pos(g, e), geo);
            th[e] = (active && j >= 0) ? src[j] : czero<T>();
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<T> w[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T fk = c == 0 ? fkx : c == 1 ? fky : az * T(k_of_pos(F::first_pos(g, e), N));
                w[e] = mul_i(cscale(th[e], fk));
            }
            F::run(w, g, lds, tw);
            if (active) {
                cx<T>* dst = A + (int64_t)(6 + c) * geo.sa + lin * N;
#pragma unroll
                for (int e = 0; e < E; ++e) dst[F::last_pos(g, e)] = w[e];
            }
        }
        F::run(th, g, lds, tw);
        if (active) {
            cx<T>* dst = A + (int64_t)9 * geo.sa + lin * N;
#pragma unroll
            for (int e = 0; e < E; ++e) dst[F::last_pos(g, e)] = th[e];
        }
    }
}

template <typename T, class CF, int NGRP, bool THETA>
__global__ __launch_bounds__(LINE_BLOCK) void k_zinv(const cx<T>* __restrict__ st, cx<T>* __restrict__ A,
                                                      const cx<T>* __restrict__ tw, Geo geo) {
    __shared__ cx<T> sm[line_lds<T, CF, LINE_BLOCK>()];
    zinv_body<T, CF, LINE_BLOCK, NGRP, THETA>(st, A, tw, geo, blockIdx.x, threadIdx.x, sm);
}

// ------------------------------------------------------------ y passes
// Tile of TL consecutive z for one (field, kx).  INV: rows = kept ky (M) ->
// all y (N); forward: all y -> kept ky.  A block of NT threads runs
// NT / (G TL) tiles side by side.
// ZN: the z length when it equals the y length N (cubic grids: compile-time
// strides), 0 for the runtime geo.n
template <typename T, class CF, int NT, bool INV, int ZN = 0>
__device__ __forceinline__ void ypass_body(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                           const cx<T>* __restrict__ tw, const Geo& geo, int64_t fs_in,
                                           int64_t fs_out, int nf, int64_t unit, int tid, cx<T>* sm) {
    // N: y points (the transform); the tile's TL columns are consecutive z of nz
    constexpr int N = CF::N, G = CF::G, TL = CF::TL, TLP = TL + 1, TT = G * TL, SG = NT / TT;
    using F = Fft<T, typename CF::P, G, INV, false, false, sizeof(T) == 4>;
    constexpr int E = F::E;
    const int nz = ZN ? ZN : geo.n, NTZ = ZN ? ztiles<(ZN ? ZN : 1), TL>() : zt_count<TL>(geo);
    const int s = tid / TT, r = tid % TT;
    const int t = r % TL, g = r / TL;
    const int64_t tile = unit * SG + s;
    const bool valid = tile < (int64_t)nf * geo.nxk * NTZ;
    const int zt = valid ? (int)(tile % NTZ) : 0;
    const int64_t rest = valid ? tile / NTZ : 0;
    const int kx = (int)(rest % geo.nxk), f = (int)(rest / geo.nxk);
    const int z = zt * TL + t;
    const bool zin = valid && z < nz;
    // kx plane strides: My nz on the A side, pb (padded) on the B / C side
    const int64_t pa = (int64_t)geo.My * nz;
    const cx<T>* src = in + f * fs_in + (int64_t)kx * (INV ? pa : geo.pb) + z;
    cx<T>* dst = out + f * fs_out + (int64_t)kx * (INV ? geo.pb : pa) + z;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = F::first_pos(g, e);
        const int row = INV ? jy_of_pos(p, geo) : p;
        v[e] = (zin && row >= 0) ? src[(int64_t)row * nz] : czero<T>();
    }
    F::run(v, g, TileLds<T, TLP>{sm + s * N * TLP + t}, tw);
    if (zin) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = F::last_pos(g, e);
            const int row = INV ? q : jy_of_pos(q, geo);
            if (row >= 0) dst[(int64_t)row * nz] = v[e];
        }
    }
}

template <typename T, class CF, bool INV, int ZN>
__global__ __launch_bounds__((CF::G * CF::TL)) void k_ypass(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                          const cx<T>* __restrict__ tw, Geo geo, int64_t fs_in,
                                                          int64_t fs_out, int nf) {
    __shared__ cx<T> sm[tile_lds<T, CF, CF::G * CF::TL>()];
    // FP64: each XCD takes a contiguous range of tiles (measured 10% faster; FP32 slightly slower)
    ypass_body<T, CF, CF::G * CF::TL, INV, ZN>(in, out, tw, geo, fs_in, fs_out, nf,
                                               sizeof(T) == 8 ? xcd_unit() : (int64_t)blockIdx.x, threadIdx.x, sm);
}

// ------------------------------------------------------------ fused x pass
// Tile of TL consecutive z at one y.  Backward x for the field pairs
// (v, i k x v) packed as one complex line each (two real transforms for the
// price of one), cross products in registers, forward x of the products
// packed two per complex line, split by Hermitian symmetry, kx <= K kept.
// SYS: 0 Navier-Stokes, 1 MHD, 2 Boussinesq (nbv: Brunt-Vaisala frequency).
// KC: the x cutoff Kx as a compile-time constant (0: read from geo), which
// lets the compiler drop the loads, selects and stores of the rows and points
// that lie wholly inside or outside the kept band.
template <typename T, class CF, int NT, int SYS, bool PPB = false, bool BLK = false, int KC = 0>
__device__ __forceinline__ void xpass_body(const cx<T>* __restrict__ Bf, cx<T>* __restrict__ Cf,
                                           const cx<T>* __restrict__ tw, const Geo& geo, int64_t unit, int tid,
                                           cx<T>* sm, T nbv = T(0)) {
    constexpr bool MHD = SYS == 1, BQ = SYS == 2;
    constexpr int N = CF::N, G = CF::G, TL = CF::TL, TLP = TL + 1, TT = G * TL, SG = NT / TT;
    using FI = Fft<T, typename CF::P, G, true, false, false, sizeof(T) == 4>;
    using FF = Fft<T, typename CF::P, G, false, true, false, sizeof(T) == 4>;
    // N: x points (the transform); tiles over y (ny) and z tiles of nz
    constexpr int E = FI::E;
    const int nz = geo.n, NTZ = zt_count<TL>(geo);
    constexpr int NP = MHD ? 6 : BQ ? 5 : 3;   // backward pairs
    constexpr int NO = MHD ? 3 : 2;            // forward packed lines
    constexpr int NOUT = MHD ? 6 : BQ ? 4 : 3; // output fields
    const int s = tid / TT, r = tid % TT;
    const int t = r % TL, g = r / TL;
    const int64_t tile = unit * SG + s;
    const bool valid = tile < (int64_t)geo.ny * NTZ;
    const int zt = valid ? (int)(tile % NTZ) : 0;
    const int y = valid ? (int)(tile / NTZ) : 0;
    const int z = zt * TL + t;
    const bool zin = valid && z < nz;
    // PPB: two LDS buffers of the block's tiles, used by alternate phases
    // (staging of a pair, transform exchanges, output staging), so that each
    // phase needs a single barrier (see Fft::run_pp).  BLK: block-padded tile
    // layout (TileBlk) instead of one pad slot per point.
    using TV = std::conditional_t<BLK, TileBlk<T, TL>, TileLds<T, TLP>>;
    constexpr int TSZ1 = BLK ? TileBlk<T, TL>::size(N) : N * TLP;   // elements of one tile
    constexpr int TSZ = SG * TSZ1;
    // LDS indices of the staging and output phases split into a per-thread
    // base and multiples of 8 (see LineLds::at) when G and the first / last
    // stage spans N / R are multiples of 8
    constexpr bool SPLIT = G % 8 == 0 && N % (8 * FI::R_FIRST) == 0 && N % (8 * FF::R_LAST) == 0;
    const TV lds{sm + s * TSZ1 + t};
    const TV lds1{sm + (PPB ? TSZ : 0) + s * TSZ1 + t};
    int ex = 0;   // LDS phases so far
    const int64_t nn = geo.pb;   // stride of one kx plane
    const int64_t off = (int64_t)y * nz + z;
    const int K = KC ? KC : geo.Kx;
    // Each kept row kx <= K of a pair (v, i k x v) is read from HBM once into
    // LDS (coalesced along z); the packed line Z = V + i W and its Hermitian
    // mirror Z(N - kx) = conj V + i conj W are then assembled from LDS.
    cx<T> v[NP][E];
    // A thread's kept rows of a pair are kx = g + i G (i < IT, kx <= K < N/2).
    // All of them are loaded at once (a fixed, predicated count, so the loads
    // are in flight together), and the next pair's loads are issued before the
    // current pair's LDS barrier and assembly, which hides their latency.
    constexpr int IT = (N / 2 - 1) / G + 1;
    // FP32 Navier-Stokes: all three pairs are loaded at the start of the tile
    constexpr bool ALLP = sizeof(T) == 4 && SYS == 0;
    constexpr int NSL = ALLP ? NP : 1;   // pair slots in registers
    cx<T> la_[NSL][IT], lb_[NSL][IT];
    auto load_pair = [&](int pi, bool zin_, int64_t off_) {
        cx<T>(&la)[IT] = la_[ALLP ? pi : 0];
        cx<T>(&lb)[IT] = lb_[ALLP ? pi : 0];
        // pairs (v_c, (i k x v)_c); Boussinesq adds (theta_x, theta_y), (theta_z, theta)
        const int fu = (BQ && pi >= 3) ? 6 + 2 * (pi - 3) : (pi / 3) * 6 + pi % 3;
        const int fw = (BQ && pi >= 3) ? fu + 1 : fu + 3;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int kx = g + i * G;
            const bool ok = zin_ && kx <= K;
            la[i] = ok ? Bf[fu * geo.sb + kx * nn + off_] : czero<T>();
            lb[i] = ok ? Bf[fw * geo.sb + kx * nn + off_] : czero<T>();
        }
    };
    if constexpr (ALLP) {
#pragma unroll
        for (int pi = 0; pi < NP; ++pi) load_pair(pi, zin, off);
    } else {
        load_pair(0, zin, off);
    }
#pragma unroll
    for (int pi = 0; pi < NP; ++pi) {
        cx<T>(&la)[IT] = la_[ALLP ? pi : 0];
        cx<T>(&lb)[IT] = lb_[ALLP ? pi : 0];
        // this tile's LDS, points 0 .. 2K+1 < N of the tile view
        const TV stage{sm + ((PPB && (ex & 1)) ? TSZ : 0) + s * TSZ1 + t};
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int kx = g + i * G;
            if (kx <= K) {
                if constexpr (SPLIT) {
                    stage.at(g, i * G) = la[i];
                    stage.at(K + 1 + g, i * G) = lb[i];
                } else {
                    stage(kx) = la[i];
                    stage(K + 1 + kx) = lb[i];
                }
            }
        }
        if (!ALLP && pi + 1 < NP) load_pair(pi + 1, zin, off);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = FI::first_pos(g, e);
            const bool lo = p <= K, hi = p >= N - K;
            // SPLIT: p = g + d with d = first_pos(0, e) a multiple of 8, so
            // kk = g + d or N - g - d splits as at() needs.  FP32 Navier-Stokes:
            // branch-free, every lane reads a valid row (row 0 for the points
            // between the kept bands) and the result is selected (fewer scalar
            // branch instructions: 1.30 -> 1.27 ms at 512^3); the others branch
            // (selecting both alternatives costs them registers: FP64 spilled,
            // MHD and Boussinesq measured 3-5% slower).
            const bool in = lo || hi;
            const int d = FI::first_pos(0, e);
            if constexpr (sizeof(T) == 4 && SYS == 0) {
                const int kk = !in ? 0 : lo ? p : N - p;
                cx<T> U, W;
                if constexpr (SPLIT) {
                    const int b0 = !in ? 0 : lo ? g : N - g, dd = !in ? 0 : lo ? d : -d;
                    U = stage.at(b0, dd);
                    W = stage.at(K + 1 + b0, dd);
                } else {
                    U = stage(kk);
                    W = stage(K + 1 + kk);
                }
                cx<T> Z = lo ? cx<T>{U.x - W.y, U.y + W.x} : cx<T>{U.x + W.y, W.x - U.y};
                if (p == 0) Z = {U.x, W.x};
                v[pi][e] = in ? Z : czero<T>();
            } else {
                const int kk = lo ? p : N - p;
                cx<T> Z = czero<T>();
                if (in) {
                    cx<T> U, W;
                    if constexpr (SPLIT) {
                        U = lo ? stage.at(g, d) : stage.at(N - g, -d);
                        W = lo ? stage.at(K + 1 + g, d) : stage.at(K + 1 + N - g, -d);
                    } else {
                        U = stage(kk);
                        W = stage(K + 1 + kk);
                    }
                    if (p == 0) Z = {U.x, W.x};
                    else if (lo) Z = {U.x - W.y, U.y + W.x};
                    else Z = {U.x + W.y, W.x - U.y};
                }
                v[pi][e] = Z;
            }
        }
        if constexpr (!PPB) __syncthreads();
        ++ex;
    }
#pragma unroll
    for (int pi = 0; pi < NP; ++pi) {
        if constexpr (PPB) {
            FI::run_pp(v[pi], g, lds, lds1, ex, tw);
            ex += FI::EXCH;
        } else {
            FI::run(v[pi], g, lds, tw);
        }
    }
    // physical space: Re = v, Im = curl v at x = last_pos(g, e)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const T ux = v[0][e].x, uy = v[1][e].x, uz = v[2][e].x;
        const T wx = v[0][e].y, wy = v[1][e].y, wz = v[2][e].y;
        T nx = uy * wz - uz * wy, ny = uz * wx - ux * wz, nz = ux * wy - uy * wx;
        if constexpr (MHD) {
            const T bx = v[3][e].x, by = v[4][e].x, bz = v[5][e].x;
            const T jx = v[3][e].y, jy = v[4][e].y, jz = v[5][e].y;
            nx += jy * bz - jz * by;
            ny += jz * bx - jx * bz;
            nz += jx * by - jy * bx;
            const T mx = uy * bz - uz * by, my = uz * bx - ux * bz, mz = ux * by - uy * bx;
            v[0][e] = {nx, ny};
            v[1][e] = {nz, mx};
            v[2][e] = {my, mz};
        } else if constexpr (BQ) {
            // buoyancy -N theta zhat joins the momentum products; the scalar's
            // term is -u . grad theta + N u_z
            const T gx = v[3][e].x, gy = v[3][e].y, gz = v[4][e].x, th = v[4][e].y;
            v[0][e] = {nx, ny};
            v[1][e] = {nz - nbv * th, nbv * uz - (ux * gx + uy * gy + uz * gz)};
        } else {
            v[0][e] = {nx, ny};
            v[1][e] = {nz, T(0)};
        }
    }
#pragma unroll
    for (int po = 0; po < NO; ++po) {
        if constexpr (PPB) {
            FF::run_pp(v[po], g, lds, lds1, ex, tw);
            ex += FF::EXCH;
        } else {
            FF::run(v[po], g, lds, tw);
        }
        const TV lo = (PPB && (ex & 1)) ? lds1 : lds;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            // with a compiled-in cutoff, points that no thread's kept row
            // kx <= K or mirror N - kx needs are neither stored nor computed
            const int d = FF::last_pos(0, e);
            if (KC && FF::R_LAST * G == N && d > K && d + G - 1 < N - K) continue;
            if constexpr (SPLIT) lo.at(g, FF::last_pos(0, e)) = v[po][e];
            else lo(FF::last_pos(g, e)) = v[po][e];
        }
        __syncthreads();
        if (zin) {
            const int fa = 2 * po, fb = 2 * po + 1;
            // rows kx = g + i G <= K: FP32 a fixed, predicated count (unrolled),
            // FP64 a loop (fewer live registers)
            auto out_row = [&](int i) {
                const int kx = g + i * G, d = i * G;
                cx<T> a, b;
                if constexpr (SPLIT) {
                    a = lo.at(g, d);
                    b = lo.at(kx == 0 ? 0 : N - g, kx == 0 ? 0 : -d);   // the mirror N - kx (0 for kx = 0)
                } else {
                    a = lo(kx);
                    b = lo(kx == 0 ? 0 : N - kx);
                }
                const cx<T> A = {T(0.5) * (a.x + b.x), T(0.5) * (a.y - b.y)};
                Cf[fa * geo.sb + kx * nn + off] = A;
                if (fb < NOUT) {
                    const cx<T> Bv = {T(0.5) * (a.y + b.y), T(-0.5) * (a.x - b.x)};
                    Cf[fb * geo.sb + kx * nn + off] = Bv;
                }
            };
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int i = 0; i < IT; ++i)
                    if (g + i * G <= K) out_row(i);
            } else {
                for (int i = 0; g + i * G <= K; ++i) out_row(i);
            }
        }
        if constexpr (!PPB) __syncthreads();
        ++ex;
    }
}

// Two tile buffers for Navier-Stokes where they fit in the 160 KB of LDS of
// a CU (for MHD the alternating views cost registers, and occupancy at 1024).
// LDS elements of one buffer of the x pass (block-padded tiles).
template <typename T, class CF, int NT> constexpr int xtile_lds() {
    return (NT / (CF::G * CF::TL)) * TileBlk<T, CF::TL>::size(CF::N);
}

template <typename T, class CF, bool MHD> constexpr bool xpass_pp() {
    return !MHD && 2 * xtile_lds<T, CF, CF::G * CF::TL>() * (int)sizeof(cx<T>) <= 160 * 1024;
}

// Two workgroups per CU for the FP32 Navier-Stokes x pass: its tile (8 lines
// of 64 threads below n = 1024, 4 lines of 128 threads at 1024) fits 128
// VGPRs, so two tiles are in flight per CU and one's loads overlap the
// other's transforms (1.52 -> 1.49 ms at 512^3 against one 16-line tile per CU).
template <typename T, int N, int SYS> constexpr bool xpass_two_per_cu() {
    return SYS == 0 && sizeof(T) == 4;
}

// Tiles per workgroup: FP64 and the other half-height FP32 tiles (Boussinesq,
// n = 1024) loop over 32 consecutive tiles, which overlaps one tile's final
// stores with the next tile's first reads (measured 11% faster for FP64
// Navier-Stokes and the FP32 Boussinesq x pass at 512^3); MHD and the FP32
// Navier-Stokes tiles take one tile (a loop costs them registers and
// occupancy).
template <typename T, class CF, int SYS> constexpr int xpass_per() {
    if constexpr (xpass_two_per_cu<T, CF::N, SYS>()) return 1;
    else return ((sizeof(T) == 8 || CF::TL < tile_lines<T>()) && xpass_pp<T, CF, SYS == 1>()) ? 32 : 1;
}

template <typename T, class CF, int SYS, int KC = 0>
__global__ __launch_bounds__((CF::G * CF::TL), (xpass_two_per_cu<T, CF::N, SYS>() ? 4 : 1)) void k_xpass(const cx<T>* __restrict__ Bf, cx<T>* __restrict__ Cf,
                                                          const cx<T>* __restrict__ tw, Geo geo, T nbv) {
    constexpr bool PPB = xpass_pp<T, CF, SYS == 1>();
    constexpr int PER = xpass_per<T, CF, SYS>();
    __shared__ cx<T> sm[(PPB ? 2 : 1) * xtile_lds<T, CF, CF::G * CF::TL>()];
    // each XCD takes a contiguous range of tiles (measured faster, most for the
    // narrow MHD tiles at n = 1024 whose rows share cache lines)
    if constexpr (PER == 1) {
        xpass_body<T, CF, CF::G * CF::TL, SYS, PPB, true, KC>(Bf, Cf, tw, geo, xcd_unit(), threadIdx.x, sm, nbv);
    } else {
        const int64_t ntl = (int64_t)geo.ny * zt_count<CF::TL>(geo);
        const int64_t u0 = xcd_unit() * PER;
        const int64_t u1 = u0 + PER < ntl ? u0 + PER : ntl;
        for (int64_t u = u0; u < u1; ++u) {
            if (u > u0) __syncthreads();   // the previous tile's last LDS reads
            xpass_body<T, CF, CF::G * CF::TL, SYS, PPB, true, KC>(Bf, Cf, tw, geo, u, threadIdx.x, sm, nbv);
        }
    }
}

// ------------------------------------------------------------ zfwd + update
// The stage arrays are distinct buffers: restrict-qualified here and in
// zfwd_lines so that loads of later modes may be issued ahead of earlier stores.
template <typename T>
__device__ __forceinline__ void rk_apply(int mode, cx<T>* __restrict__ U, cx<T>* __restrict__ V,
                                         cx<T>* __restrict__ Acc, cx<T>* __restrict__ R, T h, int64_t idx, T E, T E2,
                                         cx<T> nk) {
    if (mode == Z_RHS) {
        R[idx] = nk;
        return;
    }
    switch (mode) {
        case Z_RK4_0: {
            const cx<T> un = U[idx];
            V[idx] = {E * (un.x + T(0.5) * h * nk.x), E * (un.y + T(0.5) * h * nk.y)};
            Acc[idx] = {E2 * (un.x + (h / T(6)) * nk.x), E2 * (un.y + (h / T(6)) * nk.y)};
        } break;
        case Z_RK4_1: {
            const cx<T> un = U[idx], ac = Acc[idx];
            V[idx] = {E * un.x + T(0.5) * h * nk.x, E * un.y + T(0.5) * h * nk.y};
            Acc[idx] = {ac.x + (h / T(3)) * E * nk.x, ac.y + (h / T(3)) * E * nk.y};
        } break;
        case Z_RK4_2: {
            const cx<T> un = U[idx], ac = Acc[idx];
            V[idx] = {E2 * un.x + h * E * nk.x, E2 * un.y + h * E * nk.y};
            Acc[idx] = {ac.x + (h / T(3)) * E * nk.x, ac.y + (h / T(3)) * E * nk.y};
        } break;
        case Z_RK4_3: {
            const cx<T> ac = Acc[idx];
            U[idx] = {ac.x + (h / T(6)) * nk.x, ac.y + (h / T(6)) * nk.y};
        } break;
        case Z_RK2_0: {
            const cx<T> un = U[idx];
            V[idx] = {E2 * (un.x + h * nk.x), E2 * (un.y + h * nk.y)};
            Acc[idx] = {E2 * (un.x + T(0.5) * h * nk.x), E2 * (un.y + T(0.5) * h * nk.y)};
        } break;
        case Z_RK2_1: {
            const cx<T> ac = Acc[idx];
            U[idx] = {ac.x + T(0.5) * h * nk.x, ac.y + T(0.5) * h * nk.y};
        } break;
        default: break;
    }
}

// ANI: a non-cubic grid or box (|k|^2 not an integer): the integrating
// factors are evaluated per mode; a separate instantiation keeps the FP64 path
// out of the cubic kernels' register allocation.
template <typename T, class CF, int NT, int SYS, bool ANI = false>
__device__ __forceinline__ void zfwd_lines(const cx<T>* __restrict__ D, const cx<T>* __restrict__ tw, const Geo& geo,
                                           const RkArgs<T>& ra, cx<T>* __restrict__ U, cx<T>* __restrict__ V,
                                           cx<T>* __restrict__ Acc, cx<T>* __restrict__ R, int mode, int64_t unit,
                                           int tid, cx<T>* sm) {
    constexpr int N = CF::N, G = CF::G;
    using F = Fft<T, typename CF::P, G, false, false, false, sizeof(T) == 4>;
    constexpr int E = F::E, LPB = NT / G, LS = LineLds<T>::size(N);
    constexpr bool MHD = SYS == 1, BQ = SYS == 2;
    constexpr int NF = MHD ? 6 : BQ ? 4 : 3;
    const int l = tid / G, g = tid % G;
    const int64_t line = unit * LPB + l;
    const bool active = line < (int64_t)geo.nxk * geo.My;
    const int kx = active ? (int)(line / geo.My) : 0;
    const int jy = active ? (int)(line % geo.My) : 0;
    const int iky = ky_of_j(jy, geo);
    const LineLds<T> lds{sm + l * LS};
    const int64_t lin = (int64_t)kx * geo.My + jy;
    cx<T> v[NF][E];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const cx<T>* src = D + f * geo.sa + lin * N;
#pragma unroll
        for (int e = 0; e < E; ++e) v[f][e] = active ? src[F::first_pos(g, e)] : czero<T>();
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) F::run(v[f], g, lds, tw);
    if (!active) return;
    const T scale = T(1) / (T(geo.nx) * T(geo.ny) * T(N));
    // physical wavenumbers a_i k_i (equal to the integers on the 2 pi box)
    const T fkx = T(geo.ax) * T(kx), fky = T(geo.ay) * T(iky);
    const double kxy2 = ANI ? geo.ax * geo.ax * kx * kx + geo.ay * geo.ay * iky * iky : 0.0;
    // kx^2 + ky^2: uniform over a wavefront when a line fills whole
    // wavefronts (G >= 64), so its table entries come through scalar loads
    // into scalar registers
    const int kp2 = G >= 64 ? __builtin_amdgcn_readfirstlane(kx * kx + iky * iky) : 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = F::last_pos(g, e);
        const int j = j_of_pos(q, geo);
        if (j < 0) continue;
        const int ikz = k_of_pos(q, N);
        const T fkz = T(geo.az) * T(ikz);
        const int k2 = kx * kx + iky * iky + ikz * ikz;   // integer |k|^2: table index (2 pi box)
        const int64_t idx = lin * geo.M + j;
        cx<T> n0 = cscale(v[0][e], scale), n1 = cscale(v[1][e], scale), n2 = cscale(v[2][e], scale);
        // projection onto divergence-free fields: n - k (k . n) / |k|^2, zero at
        // k = 0 and, with spherical truncation, outside the sphere
        const bool cut = ra.sph2 >= 0 && k2 > ra.sph2;
        cx<T> o[3];
        if (k2 == 0 || cut) {
            o[0] = o[1] = o[2] = czero<T>();
        } else {
            const T ik2 = T(1) / (fkx * fkx + fky * fky + fkz * fkz);
            const cx<T> kn = {(fkx * n0.x + fky * n1.x + fkz * n2.x) * ik2, (fkx * n0.y + fky * n1.y + fkz * n2.y) * ik2};
            o[0] = {n0.x - fkx * kn.x, n0.y - fkx * kn.y};
            o[1] = {n1.x - fky * kn.x, n1.y - fky * kn.y};
            o[2] = {n2.x - fkz * kn.x, n2.y - fkz * kn.y};
        }
        if (!MHD && ra.F && kx <= ra.kf && iky <= ra.kf && -iky <= ra.kf && ikz <= ra.kf && -ikz <= ra.kf) {
            const int w = 2 * ra.kf + 1;
            const int64_t fi = ((int64_t)kx * w + (iky + ra.kf)) * w + (ikz + ra.kf);
            const int64_t fs = (int64_t)(ra.kf + 1) * w * w;
#pragma unroll
            for (int c = 0; c < 3; ++c) o[c] = cadd(o[c], ra.F[c * fs + fi]);
        }
        if (ra.lin_only) o[0] = o[1] = o[2] = czero<T>();
        // integrating factors: on the 2 pi box, for lines of whole
        // wavefronts (n >= 512), the product of the tables at kx^2 + ky^2
        // (one scalar load per line) and at kz^2 (the same few entries for
        // every line), exp(-c |k|^2) = exp(-c k_perp^2) exp(-c kz^2): a direct
        // lookup by |k|^2 scatters over the whole table, which at n = 1024
        // (1.4 MB per table) L2 does not keep and fetched again (1.55x the
        // algorithmic bytes of the MHD pass); smaller grids, whose tables stay
        // in cache, look up |k|^2 directly; on other boxes exp(-visc |k|^2 h / 2)
        // is evaluated here in FP64 and rounded once.  Loaded once per mode for
        // all components (the stage-array stores in between would otherwise
        // force reloads).
        T Eu, E2u;
        if constexpr (!ANI && G >= 64) {
            Eu = ra.E[0][kp2] * ra.E[0][ikz * ikz];
            E2u = ra.E2[0][kp2] * ra.E2[0][ikz * ikz];
        } else if constexpr (!ANI) {
            Eu = ra.E[0][k2];
            E2u = ra.E2[0][k2];
        } else {
            const double eu = exp(-0.5 * ra.visc[0] * ra.hd * (kxy2 + geo.az * geo.az * ikz * ikz));
            Eu = T(eu);
            E2u = T(eu * eu);
        }
        // the second group's factors (b, theta), loaded where they are used
        auto second_if = [&](T& Eb, T& E2b) {
            if constexpr (!ANI && G >= 64) {
                Eb = ra.E[1][kp2] * ra.E[1][ikz * ikz];
                E2b = ra.E2[1][kp2] * ra.E2[1][ikz * ikz];
            } else if constexpr (!ANI) {
                Eb = ra.E[1][k2];
                E2b = ra.E2[1][k2];
            } else {
                const double eb = exp(-0.5 * ra.visc[1] * ra.hd * (kxy2 + geo.az * geo.az * ikz * ikz));
                Eb = T(eb);
                E2b = T(eb * eb);
            }
        };
#pragma unroll
        for (int c = 0; c < 3; ++c) rk_apply(mode, U, V, Acc, R, ra.h, c * geo.sc + idx, Eu, E2u, o[c]);
        if constexpr (MHD) {
            // b: i k x F[u x b]
            const cx<T> m0 = cscale(v[3][e], scale), m1 = cscale(v[4][e], scale), m2 = cscale(v[5][e], scale);
            cx<T> b[3];
            b[0] = mul_i(cx<T>{fky * m2.x - fkz * m1.x, fky * m2.y - fkz * m1.y});
            b[1] = mul_i(cx<T>{fkz * m0.x - fkx * m2.x, fkz * m0.y - fkx * m2.y});
            b[2] = mul_i(cx<T>{fkx * m1.x - fky * m0.x, fkx * m1.y - fky * m0.y});
            if (ra.lin_only || cut) b[0] = b[1] = b[2] = czero<T>();
            T Eb, E2b;
            second_if(Eb, E2b);
#pragma unroll
            for (int c = 0; c < 3; ++c) rk_apply(mode, U, V, Acc, R, ra.h, (3 + c) * geo.sc + idx, Eb, E2b, b[c]);
        }
        if constexpr (BQ) {
            // scalar: D (-F[u . grad theta] + N w_z), its own integrating factor
            cx<T> q = cscale(v[3][e], scale);
            if (ra.lin_only || cut) q = czero<T>();
            T Eb, E2b;
            second_if(Eb, E2b);
            rk_apply(mode, U, V, Acc, R, ra.h, 3 * geo.sc + idx, Eb, E2b, q);
        }
    }
}

// SYS: 0 Navier-Stokes, 1 MHD, 2 Boussinesq.
template <typename T, class CF, int NT, int SYS, bool ANI = false>
__device__ __forceinline__ void zfwd_body(const cx<T>* __restrict__ D, const cx<T>* __restrict__ tw, const Geo& geo,
                                          const RkArgs<T>& ra, int mode, int64_t unit, int tid, cx<T>* sm) {
    zfwd_lines<T, CF, NT, SYS, ANI>(D, tw, geo, ra, ra.U, ra.V, ra.Acc, ra.R, mode, unit, tid, sm);
}

template <typename T, class CF, int SYS, bool ANI>
__global__ __launch_bounds__(LINE_BLOCK) void k_zfwd(const cx<T>* __restrict__ D, const cx<T>* __restrict__ tw,
                                                      Geo geo, RkArgs<T> ra, int mode) {
    __shared__ cx<T> sm[line_lds<T, CF, LINE_BLOCK>()];
    zfwd_body<T, CF, LINE_BLOCK, SYS, ANI>(D, tw, geo, ra, mode, blockIdx.x, threadIdx.x, sm);
}

// ------------------------------------------------------------ standalone FFTs
// Physical [nf][n][n][n] real, spectral [nf][n][n][n/2+1] complex (ABI layout).

// x, forward: two real lines packed into one complex line, split afterwards.
template <typename T, int N>
__global__ __launch_bounds__(LINE_BLOCK) void k_fftx_r2c(const T* __restrict__ in, cx<T>* __restrict__ out,
                                                          const cx<T>* __restrict__ tw, int64_t npairs) {
    using C = NCfg<N>;
    using F = Fft<T, typename C::P, C::G, false, false, false, sizeof(T) == 4>;
    constexpr int G = C::G, E = F::E, LPB = LINE_BLOCK / G, LS = LineLds<T>::size(N), NXH = N / 2 + 1;
    __shared__ cx<T> sm[LPB * LS];
    const int l = threadIdx.x / G, g = threadIdx.x % G;
    const int64_t pair = (int64_t)blockIdx.x * LPB + l;
    const bool active = pair < npairs;
    const LineLds<T> lds{sm + l * LS};
    const T* a = in + 2 * pair * N;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = F::first_pos(g, e);
        v[e] = active ? cx<T>{a[p], a[N + p]} : czero<T>();
    }
    F::run(v, g, lds, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) lds(F::last_pos(g, e)) = v[e];
    __syncthreads();
    if (!active) return;
    cx<T>* oa = out + 2 * pair * NXH;
    for (int k = g; k < NXH; k += G) {
        const cx<T> z1 = lds(k), z2 = lds(k == 0 ? 0 : N - k);
        oa[k] = {T(0.5) * (z1.x + z2.x), T(0.5) * (z1.y - z2.y)};
        oa[NXH + k] = {T(0.5) * (z1.y + z2.y), T(-0.5) * (z1.x - z2.x)};
    }
}

// x, backward: Hermitian extension of two half lines packed as A + i B.
template <typename T, int N>
__global__ __launch_bounds__(LINE_BLOCK) void k_fftx_c2r(const cx<T>* __restrict__ in, T* __restrict__ out,
                                                          const cx<T>* __restrict__ tw, int64_t npairs) {
    using C = NCfg<N>;
    using F = Fft<T, typename C::P, C::G, true, false, false, sizeof(T) == 4>;
    constexpr int G = C::G, E = F::E, LPB = LINE_BLOCK / G, LS = LineLds<T>::size(N), NXH = N / 2 + 1;
    __shared__ cx<T> sm[LPB * LS];
    const int l = threadIdx.x / G, g = threadIdx.x % G;
    const int64_t pair = (int64_t)blockIdx.x * LPB + l;
    const bool active = pair < npairs;
    const LineLds<T> lds{sm + l * LS};
    const cx<T>* ia = in + 2 * pair * NXH;
    // The pair's two half lines are contiguous: read them once, coalesced,
    // into this line's LDS, then assemble Z(p) and its Hermitian mirror there.
    static_assert(2 * NXH <= LineLds<T>::size(N), "the staged pair must fit the line's LDS");
    cx<T>* st = sm + l * LS;
    for (int k = g; k < 2 * NXH; k += G) st[k] = active ? ia[k] : czero<T>();
    __syncthreads();
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = F::first_pos(g, e);
        if (p == 0 || 2 * p == N) {
            v[e] = {st[p].x, st[NXH + p].x};
        } else if (p < NXH) {
            const cx<T> A = st[p], B = st[NXH + p];
            v[e] = {A.x - B.y, A.y + B.x};
        } else {
            const cx<T> A = st[N - p], B = st[NXH + N - p];
            v[e] = {A.x + B.y, B.x - A.y};
        }
    }
    __syncthreads();  // the transform reuses the staging area
    F::run(v, g, lds, tw);
    if (!active) return;
    T* oa = out + 2 * pair * N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = F::last_pos(g, e);
        oa[q] = v[e].x;
        oa[N + q] = v[e].y;
    }
}

// Strided complex pass over rows of stride `rs` (elements), TL consecutive
// columns per workgroup (ragged at ncols), planes of `ps` elements along
// blockIdx.y.  Used for y (rs = n/2+1) and z (rs = n (n/2+1)) of the
// standalone transforms; in == out is allowed.
template <typename T, int N, bool INV>
__global__ __launch_bounds__(NCfg<N>::G * tile_lines<T>()) void k_fft_strided(const cx<T>* in, cx<T>* out,
                                                                              const cx<T>* __restrict__ tw,
                                                                              int64_t rs, int64_t ncols, int64_t ps,
                                                                              T scale) {
    using C = NCfg<N>;
    using F = Fft<T, typename C::P, C::G, INV, false, false, sizeof(T) == 4>;
    constexpr int G = C::G, E = F::E, TL = tile_lines<T>(), TLP = TL + 1;
    __shared__ cx<T> sm[N * TLP];
    const int t = threadIdx.x % TL, g = threadIdx.x / TL;
    // Workgroups go to the 8 XCDs round-robin.  When tile rows straddle cache
    // lines (row length not a multiple of the tile), each XCD takes a
    // contiguous range of (plane, column tile) pairs so that neighbouring
    // tiles, which share those lines, meet in the same L2 (FP64 too, where it
    // measured faster for every pass).
    const int64_t nbx = gridDim.x, nbl = nbx * gridDim.y, lin = (int64_t)blockIdx.y * nbx + blockIdx.x;
    const bool xcd = nbl % 8 == 0 && (rs % TL != 0 || sizeof(T) == 8);
    const int64_t rl = xcd ? (lin % 8) * (nbl / 8) + lin / 8 : lin;
    const int64_t bx = rl % nbx, by = rl / nbx;
    const int64_t col = bx * TL + t;
    const bool cin = col < ncols;
    const int64_t base = by * ps + col;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cin ? in[base + F::first_pos(g, e) * rs] : czero<T>();
    F::run(v, g, TileLds<T, TLP>{sm + t}, tw);
    if (cin) {
#pragma unroll
        for (int e = 0; e < E; ++e) out[base + F::last_pos(g, e) * rs] = cscale(v[e], scale);
    }
}

// ------------------------------------------------------------ mode-pruned transforms
// 3D r2c / c2r restricted to the box kx in [0, m), ky, kz in [0, m) U [N-m, N)
// (compact index j < m <-> position j, j >= m <-> position j + N - 2m), laid
// out [field][jz][jy][kx] (kx fastest).  Used by the spectral layers of the
// neural operator.

// x, forward, keep kx < m: out [lines][m]
template <typename T, int N>
__global__ __launch_bounds__(LINE_BLOCK) void k_fftx_r2c_m(const T* __restrict__ in, cx<T>* __restrict__ out,
                                                            const cx<T>* __restrict__ tw, int64_t npairs, int m) {
    using C = NCfg<N>;
    using F = Fft<T, typename C::P, C::G, false, false, false, sizeof(T) == 4>;
    constexpr int G = C::G, E = F::E, LPB = LINE_BLOCK / G, LS = LineLds<T>::size(N);
    __shared__ cx<T> sm[LPB * LS];
    const int l = threadIdx.x / G, g = threadIdx.x % G;
    const int64_t pair = (int64_t)blockIdx.x * LPB + l;
    const bool active = pair < npairs;
    const LineLds<T> lds{sm + l * LS};
    const T* a = in + 2 * pair * N;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = F::first_pos(g, e);
        v[e] = active ? cx<T>{a[p], a[N + p]} : czero<T>();
    }
    F::run(v, g, lds, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) lds(F::last_pos(g, e)) = v[e];
    __syncthreads();
    if (!active) return;
    cx<T>* oa = out + 2 * pair * m;
    for (int k = g; k < m; k += G) {
        const cx<T> z1 = lds(k), z2 = lds(k == 0 ? 0 : N - k);
        oa[k] = {T(0.5) * (z1.x + z2.x), T(0.5) * (z1.y - z2.y)};
        oa[m + k] = {T(0.5) * (z1.y + z2.y), T(-0.5) * (z1.x - z2.x)};
    }
}

// x, backward from kx < m (Hermitian extension, imaginary part of kx = 0 dropped)
template <typename T, int N>
__global__ __launch_bounds__(LINE_BLOCK) void k_fftx_c2r_m(const cx<T>* __restrict__ in, T* __restrict__ out,
                                                            const cx<T>* __restrict__ tw, int64_t npairs, int m) {
    using C = NCfg<N>;
    using F = Fft<T, typename C::P, C::G, true, false, false, sizeof(T) == 4>;
    constexpr int G = C::G, E = F::E, LPB = LINE_BLOCK / G, LS = LineLds<T>::size(N);
    __shared__ cx<T> sm[LPB * LS];
    const int l = threadIdx.x / G, g = threadIdx.x % G;
    const int64_t pair = (int64_t)blockIdx.x * LPB + l;
    const bool active = pair < npairs;
    const LineLds<T> lds{sm + l * LS};
    const cx<T>* ia = in + 2 * pair * m;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = F::first_pos(g, e);
        cx<T> Z = czero<T>();
        if (active) {
            if (p == 0) {
                Z = {ia[0].x, ia[m].x};
            } else if (p < m) {
                const cx<T> A = ia[p], B = ia[m + p];
                Z = {A.x - B.y, A.y + B.x};
            } else if (p > N - m) {
                const cx<T> A = ia[N - p], B = ia[m + N - p];
                Z = {A.x + B.y, B.x - A.y};
            }
        }
        v[e] = Z;
    }
    F::run(v, g, lds, tw);
    if (!active) return;
    T* oa = out + 2 * pair * N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = F::last_pos(g, e);
        oa[q] = v[e].x;
        oa[N + q] = v[e].y;
    }
}

// Strided pass over TL consecutive columns of a plane (blockIdx.y); rows are
// either all N positions (row p at p * rs) or the 2m retained ones (row j at
// j * rs), separately for input (PIN) and output (POUT).
template <typename T, int N, bool INV, bool PIN, bool POUT>
__global__ __launch_bounds__(NCfg<N>::G * tile_lines<T>()) void k_fft_cols_m(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ tw, int64_t ncols, int64_t rs_in,
    int64_t ps_in, int64_t rs_out, int64_t ps_out, int m, T scale) {
    using C = NCfg<N>;
    using F = Fft<T, typename C::P, C::G, INV, false, false, sizeof(T) == 4>;
    constexpr int G = C::G, E = F::E, TL = tile_lines<T>(), TLP = TL + 1;
    __shared__ cx<T> sm[N * TLP];
    const int t = threadIdx.x % TL, g = threadIdx.x / TL;
    const int64_t col = (int64_t)blockIdx.x * TL + t;
    const bool cin = col < ncols;
    const cx<T>* src = in + (int64_t)blockIdx.y * ps_in + col;
    cx<T>* dst = out + (int64_t)blockIdx.y * ps_out + col;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = F::first_pos(g, e);
        const int row = PIN ? (p < m ? p : (p >= N - m ? p - (N - 2 * m) : -1)) : p;
        v[e] = (cin && row >= 0) ? src[row * rs_in] : czero<T>();
    }
    F::run(v, g, TileLds<T, TLP>{sm + t}, tw);
    if (cin) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = F::last_pos(g, e);
            const int row = POUT ? (q < m ? q : (q >= N - m ? q - (N - 2 * m) : -1)) : q;
            if (row >= 0) dst[row * rs_out] = cscale(v[e], scale);
        }
    }
}

// ------------------------------------------------------------ Gross-Pitaevskii
// The wavefunction psi of eq. gpe is complex: its coefficients fill the whole
// spectrum and every axis is a full c2c axis.  The compact state is
// [jx][jy][jz] over the kept cube |k_i| <= K (K = ceil(n/4) - 1: 4K < n, no
// aliasing of the cubic product); geo.nxk = M.  One right-hand side is
//   zinv   state (kept kz)     -> backward z                        -> A
//   yinv   (ypass_body, 1 field)                                    -> B
//   xpass  B (kept kx rows)    -> backward x, |psi|^2 psi, forward x,
//                                 keep kept kx                        -> C
//   yfwd   (ypass_body, 1 field)                                    -> D
//   zfwd   D                   -> forward z, keep kept kz, -i beta / n^3,
//                                 Lawson RK stage with exp(-i alpha |k|^2 h / 2)

template <typename T, class CF, int NT>
__device__ __forceinline__ void zinv_gpe_body(const cx<T>* __restrict__ st, cx<T>* __restrict__ A,
                                              const cx<T>* __restrict__ tw, const Geo& geo, int64_t unit, int tid,
                                              cx<T>* sm) {
    constexpr int N = CF::N, G = CF::G;
    using F = Fft<T, typename CF::P, G, true, false, sizeof(T) == 8 && G <= 64, sizeof(T) == 4>;
    constexpr int E = F::E, LPB = NT / G, LS = LineLds<T>::size(N);
    const int l = tid / G, g = tid % G;
    const int64_t line = unit * LPB + l;
    const bool active = line < (int64_t)geo.nxk * geo.My;
    const LineLds<T> lds{sm + l * LS};
    const cx<T>* src = st + (active ? line : 0) * geo.M;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = j_of_pos(F::first_pos(g, e), geo);
        v[e] = (active && j >= 0) ? src[j] : czero<T>();
    }
    F::run(v, g, lds, tw);
    if (active) {
        cx<T>* dst = A + line * N;
#pragma unroll
        for (int e = 0; e < E; ++e) dst[F::last_pos(g, e)] = v[e];
    }
}

template <typename T, class CF>
__global__ __launch_bounds__(LINE_BLOCK) void k_zinv_gpe(const cx<T>* __restrict__ st, cx<T>* __restrict__ A,
                                                          const cx<T>* __restrict__ tw, Geo geo) {
    __shared__ cx<T> sm[line_lds<T, CF, LINE_BLOCK>()];
    zinv_gpe_body<T, CF, LINE_BLOCK>(st, A, tw, geo, blockIdx.x, threadIdx.x, sm);
}

// Tile of TL consecutive z at one y: the kept kx rows of psi (read straight
// from HBM, TL consecutive z per row), backward x, the cubic product
// |psi|^2 psi at each point, forward x, kept rows written back.
template <typename T, class CF, int NT>
__device__ __forceinline__ void xpass_gpe_body(const cx<T>* __restrict__ Bf, cx<T>* __restrict__ Cf,
                                               const cx<T>* __restrict__ tw, const Geo& geo, int64_t unit, int tid,
                                               cx<T>* sm) {
    constexpr int N = CF::N, G = CF::G, TL = CF::TL, TT = G * TL, SG = NT / TT;
    using FI = Fft<T, typename CF::P, G, true, false, false, sizeof(T) == 4>;
    using FF = Fft<T, typename CF::P, G, false, true, false, sizeof(T) == 4>;
    constexpr int E = FI::E;
    const int nz = geo.n, NTZ = zt_count<TL>(geo);
    const int s = tid / TT, r = tid % TT;
    const int t = r % TL, g = r / TL;
    const int64_t tile = unit * SG + s;
    const bool valid = tile < (int64_t)geo.ny * NTZ;
    const int zt = valid ? (int)(tile % NTZ) : 0;
    const int y = valid ? (int)(tile / NTZ) : 0;
    const int z = zt * TL + t;
    const bool zin = valid && z < nz;
    // two LDS buffers used by alternate exchanges: one barrier per exchange
    constexpr int TSZ1 = TileBlk<T, TL>::size(N), TSZ = SG * TSZ1;
    const TileBlk<T, TL> lds0{sm + s * TSZ1 + t}, lds1{sm + TSZ + s * TSZ1 + t};
    const int64_t nn = geo.pb, off = (int64_t)y * nz + z;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = jx_of_pos(FI::first_pos(g, e), geo);
        v[e] = (zin && j >= 0) ? Bf[j * nn + off] : czero<T>();
    }
    FI::run_pp(v, g, lds0, lds1, 0, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const T a2 = v[e].x * v[e].x + v[e].y * v[e].y;
        v[e] = {a2 * v[e].x, a2 * v[e].y};
    }
    FF::run_pp(v, g, lds0, lds1, FI::EXCH, tw);
    if (zin) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = jx_of_pos(FF::last_pos(g, e), geo);
            if (j >= 0) Cf[j * nn + off] = v[e];
        }
    }
}

// Half-height tiles (8 lines FP32, 4 FP64) so that the two exchange buffers
// of a block fit twice per CU.
template <typename T, int N>
using GpeXCfg = KCfg<typename NCfg<N>::P, NCfg<N>::G, tile_lines<T>() / 2>;

template <typename T, class CF>
__global__ __launch_bounds__((CF::G * CF::TL)) void k_xpass_gpe(const cx<T>* __restrict__ Bf, cx<T>* __restrict__ Cf,
                                                               const cx<T>* __restrict__ tw, Geo geo) {
    __shared__ cx<T> sm[2 * xtile_lds<T, CF, CF::G * CF::TL>()];
    xpass_gpe_body<T, CF, CF::G * CF::TL>(Bf, Cf, tw, geo, xcd_unit(), threadIdx.x, sm);
}

// Lawson RK stage update with complex integrating factors (the arithmetic of
// rk_apply with E, E2 complex).
template <typename T>
__device__ __forceinline__ void rk_apply_cx(int mode, cx<T>* __restrict__ U, cx<T>* __restrict__ V,
                                            cx<T>* __restrict__ Acc, cx<T>* __restrict__ R, T h, int64_t idx, cx<T> E,
                                            cx<T> E2, cx<T> nk) {
    if (mode == Z_RHS) {
        R[idx] = nk;
        return;
    }
    switch (mode) {
        case Z_RK4_0: {
            const cx<T> un = U[idx];
            V[idx] = cmul(E, cadd(un, cscale(nk, T(0.5) * h)));
            Acc[idx] = cmul(E2, cadd(un, cscale(nk, h / T(6))));
        } break;
        case Z_RK4_1: {
            const cx<T> un = U[idx], ac = Acc[idx], en = cmul(E, nk);
            V[idx] = cadd(cmul(E, un), cscale(nk, T(0.5) * h));
            Acc[idx] = cadd(ac, cscale(en, h / T(3)));
        } break;
        case Z_RK4_2: {
            const cx<T> un = U[idx], ac = Acc[idx], en = cmul(E, nk);
            V[idx] = cadd(cmul(E2, un), cscale(en, h));
            Acc[idx] = cadd(ac, cscale(en, h / T(3)));
        } break;
        case Z_RK4_3: {
            const cx<T> ac = Acc[idx];
            U[idx] = cadd(ac, cscale(nk, h / T(6)));
        } break;
        case Z_RK2_0: {
            const cx<T> un = U[idx];
            V[idx] = cmul(E2, cadd(un, cscale(nk, h)));
            Acc[idx] = cmul(E2, cadd(un, cscale(nk, T(0.5) * h)));
        } break;
        case Z_RK2_1: {
            const cx<T> ac = Acc[idx];
            U[idx] = cadd(ac, cscale(nk, T(0.5) * h));
        } break;
        default: break;
    }
}

template <typename T, class CF, int NT, bool ANI>
__device__ __forceinline__ void zfwd_gpe_lines(const cx<T>* __restrict__ D, const cx<T>* __restrict__ tw,
                                               const Geo& geo, const RkArgs<T>& ra, cx<T>* __restrict__ U,
                                               cx<T>* __restrict__ V, cx<T>* __restrict__ Acc, cx<T>* __restrict__ R,
                                               int mode, int64_t unit, int tid, cx<T>* sm) {
    constexpr int N = CF::N, G = CF::G;
    using F = Fft<T, typename CF::P, G, false, false, false, sizeof(T) == 4>;
    constexpr int E = F::E, LPB = NT / G, LS = LineLds<T>::size(N);
    const int l = tid / G, g = tid % G;
    const int64_t line = unit * LPB + l;
    const bool active = line < (int64_t)geo.nxk * geo.My;
    const int jx = active ? (int)(line / geo.My) : 0;
    const int jy = active ? (int)(line % geo.My) : 0;
    const int ikx = kx_of_j(jx, geo), iky = ky_of_j(jy, geo);
    const LineLds<T> lds{sm + l * LS};
    cx<T> v[E];
    const cx<T>* src = D + (active ? line : 0) * N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = active ? src[F::first_pos(g, e)] : czero<T>();
    F::run(v, g, lds, tw);
    if (!active) return;
    // -i beta F[|psi|^2 psi] with the forward scale 1/(nx ny nz)
    const T sb = ra.beta / (T(geo.nx) * T(geo.ny) * T(N));
    const double kxy2 = ANI ? geo.ax * geo.ax * ikx * ikx + geo.ay * geo.ay * iky * iky : 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = F::last_pos(g, e);
        const int j = j_of_pos(q, geo);
        if (j < 0) continue;
        const int ikz = k_of_pos(q, N);
        const int k2 = ikx * ikx + iky * iky + ikz * ikz;
        cx<T> nk = {sb * v[e].y, -sb * v[e].x};
        if (ra.lin_only) nk = czero<T>();
        cx<T> Ef, E2f;
        if constexpr (!ANI) {
            Ef = ra.Ec[k2];
            E2f = ra.E2c[k2];
        } else {   // exp(-i alpha |k|^2 h / 2) in FP64, rounded once
            const double a = ra.visc[0] * ra.hd * (kxy2 + geo.az * geo.az * ikz * ikz);
            double sn, cs, sn2, cs2;
            sincos(0.5 * a, &sn, &cs);
            sincos(a, &sn2, &cs2);
            Ef = {T(cs), T(-sn)};
            E2f = {T(cs2), T(-sn2)};
        }
        rk_apply_cx(mode, U, V, Acc, R, ra.h, line * geo.M + j, Ef, E2f, nk);
    }
}

template <typename T, class CF, bool ANI>
__global__ __launch_bounds__(LINE_BLOCK) void k_zfwd_gpe(const cx<T>* __restrict__ D, const cx<T>* __restrict__ tw,
                                                          Geo geo, RkArgs<T> ra, int mode) {
    __shared__ cx<T> sm[line_lds<T, CF, LINE_BLOCK>()];
    zfwd_gpe_lines<T, CF, LINE_BLOCK, ANI>(D, tw, geo, ra, ra.U, ra.V, ra.Acc, ra.R, mode, blockIdx.x, threadIdx.x,
                                           sm);
}

// Contiguous complex lines of N points, one line per G threads: the x pass of
// the standalone c2c transforms (in == out allowed).
template <typename T, int N, bool INV>
__global__ __launch_bounds__(LINE_BLOCK) void k_fft_lines(const cx<T>* in, cx<T>* out, const cx<T>* __restrict__ tw,
                                                          int64_t nlines, T scale) {
    using C = NCfg<N>;
    using F = Fft<T, typename C::P, C::G, INV, false, false, sizeof(T) == 4>;
    constexpr int G = C::G, E = F::E, LPB = LINE_BLOCK / G, LS = LineLds<T>::size(N);
    __shared__ cx<T> sm[LPB * LS];
    const int l = threadIdx.x / G, g = threadIdx.x % G;
    const int64_t line = (int64_t)blockIdx.x * LPB + l;
    const bool active = line < nlines;
    const cx<T>* a = in + (active ? line : 0) * N;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = active ? a[F::first_pos(g, e)] : czero<T>();
    F::run(v, g, LineLds<T>{sm + l * LS}, tw);
    if (!active) return;
    cx<T>* o = out + line * N;
#pragma unroll
    for (int e = 0; e < E; ++e) o[F::last_pos(g, e)] = cscale(v[e], scale);
}

// ------------------------------------------------------------ launchers
inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <typename T, int N>
struct Impl {
    // the plan's table of N-th roots of unity (one per distinct axis length)
    static const void* twid(const pst_plan* P) {
        return P->geo.n == N ? P->tw : P->geo.ny == N ? P->twy : P->twx;
    }
    using C = NCfg<N>;
    static constexpr int TL = tile_lines<T>();
    static constexpr int TB = C::G * TL;

    using LC = LineCfg<T, N>;
    using TC = TileCfg<T, N>;

    static void zinv(pst_plan* P, const void* st) {
        KTimer tm(P, PST_K_ZINV);
        const Geo& g = P->geo;
        const unsigned nb = (unsigned)line_units<LC, LINE_BLOCK>(g);
        if (P->p.solver == PST_GPE)
            hipLaunchKernelGGL((k_zinv_gpe<T, LC>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream, (const cx<T>*)st,
                               (cx<T>*)P->A, (const cx<T>*)twid(P), g);
        else if (P->p.solver == PST_MHD)
            hipLaunchKernelGGL((k_zinv<T, LC, 2, false>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream, (const cx<T>*)st,
                               (cx<T>*)P->A, (const cx<T>*)twid(P), g);
        else if (P->p.solver == PST_BOUSSINESQ)
            hipLaunchKernelGGL((k_zinv<T, LC, 1, true>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream, (const cx<T>*)st,
                               (cx<T>*)P->A, (const cx<T>*)twid(P), g);
        else
            hipLaunchKernelGGL((k_zinv<T, LC, 1, false>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream, (const cx<T>*)st,
                               (cx<T>*)P->A, (const cx<T>*)twid(P), g);
    }
    static void yinv(pst_plan* P) {
        KTimer tm(P, PST_K_YINV);
        const Geo& g = P->geo;
        const unsigned nb = (unsigned)ytile_units<TC, TC::G * TC::TL>(g, P->nfin);
        if (g.n == N)   // cubic: compile-time z strides
            hipLaunchKernelGGL((k_ypass<T, TC, true, N>), dim3(nb), dim3(TC::G * TC::TL), 0, P->stream,
                               (const cx<T>*)P->A, (cx<T>*)P->B, (const cx<T>*)twid(P), g, g.sa, g.sb, P->nfin);
        else
            hipLaunchKernelGGL((k_ypass<T, TC, true, 0>), dim3(nb), dim3(TC::G * TC::TL), 0, P->stream,
                               (const cx<T>*)P->A, (cx<T>*)P->B, (const cx<T>*)twid(P), g, g.sa, g.sb, P->nfin);
    }
    static void xpass(pst_plan* P) {
        KTimer tm(P, PST_K_XPASS);
        const Geo& g = P->geo;
        if (P->p.solver == PST_GPE) {
            using GC = GpeXCfg<T, N>;
            constexpr int GB = GC::G * GC::TL;
            hipLaunchKernelGGL((k_xpass_gpe<T, GC>), dim3((unsigned)xtile_units<GC, GB>(g)), dim3(GB), 0, P->stream,
                               (const cx<T>*)P->B, (cx<T>*)P->C, (const cx<T>*)twid(P), g);
        } else if (P->p.solver == PST_MHD) {
            using XC = XCfg<T, N, true>;
            xpass_launch<XC, 1>(P, dim3((unsigned)xtile_units<XC, XC::G * XC::TL>(g)), T(0));
        } else if (P->p.solver == PST_BOUSSINESQ) {
            // five backward pairs: the MHD tile (half the lines) keeps them in registers
            using XC = XCfg<T, N, true>;
            constexpr int per = xpass_per<T, XC, 2>();
            xpass_launch<XC, 2>(P, dim3(cdiv(xtile_units<XC, XC::G * XC::TL>(g), per)), (T)P->p.nbv);
        } else {
            using XC = XCfg<T, N, false>;
            constexpr int per = xpass_per<T, XC, 0>();
            xpass_launch<XC, 0>(P, dim3(cdiv(xtile_units<XC, XC::G * XC::TL>(g), per)), T(0));
        }
    }
    // The 2/3-rule cutoff of an n-point x axis (the largest K with 3K < n) is
    // compiled into the kernel; other cutoffs take the runtime form, and so
    // does the FP64 Navier-Stokes pass at n = 1024 (its fixed-cutoff form
    // spills registers).
    template <class XC, int SYS>
    static void xpass_launch(pst_plan* P, dim3 grid, T nbv) {
        constexpr int K23 = (N + 2) / 3 - 1;
        constexpr bool FIX = !(sizeof(T) == 8 && N >= 1024 && SYS == 0);
        const dim3 block(XC::G * XC::TL);
        if (FIX && P->geo.Kx == K23)
            hipLaunchKernelGGL((k_xpass<T, XC, SYS, FIX ? K23 : 0>), grid, block, 0, P->stream, (const cx<T>*)P->B,
                               (cx<T>*)P->C, (const cx<T>*)twid(P), P->geo, nbv);
        else
            hipLaunchKernelGGL((k_xpass<T, XC, SYS>), grid, block, 0, P->stream, (const cx<T>*)P->B, (cx<T>*)P->C,
                               (const cx<T>*)twid(P), P->geo, nbv);
    }
    static void yfwd(pst_plan* P) {
        KTimer tm(P, PST_K_YFWD);
        const Geo& g = P->geo;
        const unsigned nb = (unsigned)ytile_units<TC, TC::G * TC::TL>(g, P->nfout);
        if (g.n == N)
            hipLaunchKernelGGL((k_ypass<T, TC, false, N>), dim3(nb), dim3(TC::G * TC::TL), 0, P->stream,
                               (const cx<T>*)P->C, (cx<T>*)P->A, (const cx<T>*)twid(P), g, g.sb, g.sa, P->nfout);
        else
            hipLaunchKernelGGL((k_ypass<T, TC, false, 0>), dim3(nb), dim3(TC::G * TC::TL), 0, P->stream,
                               (const cx<T>*)P->C, (cx<T>*)P->A, (const cx<T>*)twid(P), g, g.sb, g.sa, P->nfout);
    }
    static void zfwd(pst_plan* P, int mode, void* rhs_out) {
        KTimer tm(P, PST_K_ZFWD);
        const Geo& g = P->geo;
        RkArgs<T> ra;
        ra.U = (cx<T>*)P->U;
        ra.V = (cx<T>*)P->V;
        ra.Acc = (cx<T>*)P->Acc;
        ra.R = (cx<T>*)rhs_out;
        for (int i = 0; i < 2; ++i) {
            ra.E[i] = (const T*)P->Etab[i];
            ra.E2[i] = (const T*)P->E2tab[i];
        }
        ra.h = (T)P->p.dt;
        ra.F = (const cx<T>*)P->force;
        ra.kf = P->kf;
        ra.lin_only = (P->p.flags & PST_FLAG_LINEAR_ONLY) ? 1 : 0;
        ra.sph2 = P->p.dealias == PST_DEALIAS_SPHERE ? g.K * g.K : -1;
        ra.Ec = (const cx<T>*)P->Etab[0];
        ra.E2c = (const cx<T>*)P->E2tab[0];
        ra.beta = (T)P->p.beta;
        ra.visc[0] = P->p.solver == PST_GPE ? P->p.alpha : P->p.nu;
        ra.visc[1] = P->p.eta;
        ra.hd = P->p.dt;
        if (g.aniso) zfwd_launch<true>(P, ra, mode);
        else zfwd_launch<false>(P, ra, mode);
    }
    template <bool ANI>
    static void zfwd_launch(pst_plan* P, const RkArgs<T>& ra, int mode) {
        const Geo& g = P->geo;
        const unsigned nb = (unsigned)line_units<LC, LINE_BLOCK>(g);
        if (P->p.solver == PST_GPE)
            hipLaunchKernelGGL((k_zfwd_gpe<T, LC, ANI>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream,
                               (const cx<T>*)P->A, (const cx<T>*)twid(P), g, ra, mode);
        else if (P->p.solver == PST_MHD)
            hipLaunchKernelGGL((k_zfwd<T, LC, 1, ANI>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream, (const cx<T>*)P->A,
                               (const cx<T>*)twid(P), g, ra, mode);
        else if (P->p.solver == PST_BOUSSINESQ)
            hipLaunchKernelGGL((k_zfwd<T, LC, 2, ANI>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream, (const cx<T>*)P->A,
                               (const cx<T>*)twid(P), g, ra, mode);
        else
            hipLaunchKernelGGL((k_zfwd<T, LC, 0, ANI>), dim3(nb), dim3(LINE_BLOCK), 0, P->stream, (const cx<T>*)P->A,
                               (const cx<T>*)twid(P), g, ra, mode);
    }
    // One axis of the standalone 3D transforms (the runtime composes x, y, z
    // with each axis's own n).  x: nlines contiguous lines of N points (r2c /
    // c2r pack two real lines per complex transform: nlines is even).
    static void fftx_r2c(pst_plan* P, const void* in, void* out, int64_t nlines) {
        KTimer tm(P, PST_K_FFTX);
        const int64_t npairs = nlines / 2;
        hipLaunchKernelGGL((k_fftx_r2c<T, N>), dim3(cdiv(npairs, LINE_BLOCK / C::G)), dim3(LINE_BLOCK), 0,
                           P->stream, (const T*)in, (cx<T>*)out, (const cx<T>*)twid(P), npairs);
    }
    static void fftx_c2r(pst_plan* P, const void* in, void* out, int64_t nlines) {
        KTimer tm(P, PST_K_FFTX);
        const int64_t npairs = nlines / 2;
        hipLaunchKernelGGL((k_fftx_c2r<T, N>), dim3(cdiv(npairs, LINE_BLOCK / C::G)), dim3(LINE_BLOCK), 0,
                           P->stream, (const cx<T>*)in, (T*)out, (const cx<T>*)twid(P), npairs);
    }
    static void fftx_c2c(pst_plan* P, const void* in, void* out, int64_t nlines, int inverse) {
        KTimer tm(P, PST_K_FFTX);
        if (inverse)
            hipLaunchKernelGGL((k_fft_lines<T, N, true>), dim3(cdiv(nlines, LINE_BLOCK / C::G)), dim3(LINE_BLOCK), 0,
                               P->stream, (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)twid(P), nlines, T(1));
        else
            hipLaunchKernelGGL((k_fft_lines<T, N, false>), dim3(cdiv(nlines, LINE_BLOCK / C::G)), dim3(LINE_BLOCK), 0,
                               P->stream, (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)twid(P), nlines, T(1));
    }
    // y or z: N-point complex transforms down columns of stride rs, ncols
    // consecutive columns per plane, nplanes planes ps apart, times scale.
    static void fft_cols(pst_plan* P, const void* in, void* out, int64_t rs, int64_t ncols, int64_t ps,
                         int64_t nplanes, int inverse, double scale, int kind) {
        KTimer tm(P, kind);
        if (inverse)
            hipLaunchKernelGGL((k_fft_strided<T, N, true>), dim3(cdiv(ncols, TL), (unsigned)nplanes), dim3(TB), 0,
                               P->stream, (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)twid(P), rs, ncols, ps, T(scale));
        else
            hipLaunchKernelGGL((k_fft_strided<T, N, false>), dim3(cdiv(ncols, TL), (unsigned)nplanes), dim3(TB), 0,
                               P->stream, (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)twid(P), rs, ncols, ps, T(scale));
    }

    // Mode-pruned transforms.  Workspace `tmp`: t1 = nf N N m complex ([nf][z][y][kx < m],
    // the x-transformed lines) followed by t2 = nf N 2m m ([nf][z][jy][kx]).
    static void modes_yz_fwd(pst_plan* P, void* out, int nf, int m, void* tmp) {
        const int64_t m2 = 2 * m;
        cx<T>* t1 = (cx<T>*)tmp;
        cx<T>* t2 = t1 + (int64_t)nf * N * N * m;
        {
            KTimer tm(P, PST_K_FFTY);
            hipLaunchKernelGGL((k_fft_cols_m<T, N, false, false, true>), dim3(cdiv(m, TL), (unsigned)(nf * N)),
                               dim3(TB), 0, P->stream, t1, t2, (const cx<T>*)twid(P), (int64_t)m, (int64_t)m,
                               (int64_t)N * m, (int64_t)m, m2 * m, m, T(1));
        }
        {
            KTimer tm(P, PST_K_FFTZ);
            const T s = T(1) / (T(N) * T(N) * T(N));
            hipLaunchKernelGGL((k_fft_cols_m<T, N, false, false, true>), dim3(cdiv(m2 * m, TL), (unsigned)nf),
                               dim3(TB), 0, P->stream, t2, (cx<T>*)out, (const cx<T>*)twid(P), m2 * m, m2 * m,
                               (int64_t)N * m2 * m, m2 * m, m2 * m2 * m, m, s);
        }
    }
    static void modes_yz_inv(pst_plan* P, const void* in, int nf, int m, void* tmp) {
        const int64_t m2 = 2 * m;
        cx<T>* t1 = (cx<T>*)tmp;
        cx<T>* t2 = t1 + (int64_t)nf * N * N * m;
        {
            KTimer tm(P, PST_K_FFTZ);
            hipLaunchKernelGGL((k_fft_cols_m<T, N, true, true, false>), dim3(cdiv(m2 * m, TL), (unsigned)nf),
                               dim3(TB), 0, P->stream, (const cx<T>*)in, t2, (const cx<T>*)twid(P), m2 * m, m2 * m,
                               m2 * m2 * m, m2 * m, (int64_t)N * m2 * m, m, T(1));
        }
        {
            KTimer tm(P, PST_K_FFTY);
            hipLaunchKernelGGL((k_fft_cols_m<T, N, true, true, false>), dim3(cdiv(m, TL), (unsigned)(nf * N)),
                               dim3(TB), 0, P->stream, t2, t1, (const cx<T>*)twid(P), (int64_t)m, (int64_t)m, m2 * m,
                               (int64_t)m, (int64_t)N * m, m, T(1));
        }
    }
    static void fft_r2c_modes(pst_plan* P, const void* in, void* out, int nf, int m, void* tmp) {
        const int64_t npairs = (int64_t)nf * N * N / 2;
        {
            KTimer tm(P, PST_K_FFTX);
            hipLaunchKernelGGL((k_fftx_r2c_m<T, N>), dim3(cdiv(npairs, LINE_BLOCK / C::G)), dim3(LINE_BLOCK), 0,
                               P->stream, (const T*)in, (cx<T>*)tmp, (const cx<T>*)twid(P), npairs, m);
        }
        modes_yz_fwd(P, out, nf, m, tmp);
    }
    static void fft_c2r_modes(pst_plan* P, const void* in, void* out, int nf, int m, void* tmp) {
        const int64_t npairs = (int64_t)nf * N * N / 2;
        modes_yz_inv(P, in, nf, m, tmp);
        {
            KTimer tm(P, PST_K_FFTX);
            hipLaunchKernelGGL((k_fftx_c2r_m<T, N>), dim3(cdiv(npairs, LINE_BLOCK / C::G)), dim3(LINE_BLOCK), 0,
                               P->stream, (const cx<T>*)tmp, (T*)out, (const cx<T>*)twid(P), npairs, m);
        }
    }

    static const Launchers* get() {
        static Launchers L = [] {
            Launchers l{};
            l.n = N;
            for (int i = 0; i < 4; ++i) l.radices[i] = i < C::P::S ? C::P::r[i] : 0;
            l.tile_lines = TL;
            l.zinv = &zinv;
            l.yinv = &yinv;
            l.xpass = &xpass;
            l.yfwd = &yfwd;
            l.zfwd = &zfwd;
            l.fftx_r2c = &fftx_r2c;
            l.fftx_c2r = &fftx_c2r;
            l.fftx_c2c = &fftx_c2c;
            l.fft_cols = &fft_cols;
            l.fft_r2c_modes = &fft_r2c_modes;
            l.fft_c2r_modes = &fft_c2r_modes;
            l.modes_yz_fwd = &modes_yz_fwd;
            l.modes_yz_inv = &modes_yz_inv;
            return l;
        }();
        return &L;
    }
};

}  // namespace pst

#define PST_INSTANTIATE_N(NVAL)                                                          \
    namespace pst {                                                                      \
    const Launchers* launchers_n##NVAL(int precision) {                                  \
        return precision == PST_FP64 ? Impl<double, NVAL>::get() : Impl<float, NVAL>::get(); \
    }                                                                                    \
    }
