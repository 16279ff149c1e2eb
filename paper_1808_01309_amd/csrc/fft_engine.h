// Device-side FFT engine for gfx950: Stockham autosort transforms of one
// line of n complex points held in registers by G cooperating threads, with
// the data exchanged between radix stages through LDS.
//
// A line of length N = R_0 R_1 ... R_{S-1} is split over G threads; every
// thread holds E = N / G points.  Stage s (radix R, span NS = R_0...R_{s-1})
// performs the N / R butterflies b = 0 .. N/R - 1, thread g owning
// b = g + i G (i < E / R).  Butterfly b reads x[b + r N/R], multiplies by the
// twiddles w^{r (b mod NS) N / (NS R)} (w = exp(-+ 2 pi i / N)), applies an
// R-point DFT and writes y[(b / NS) NS R + (b mod NS) + r NS] (Stockham,
// natural order out).  The first stage's reads and the last stage's writes
// are both at b + r N/R, so callers load straight from and store straight to
// global memory; only the interior stages go through LDS.
//
// The forward transform uses sign -, the inverse sign +; neither scales.
// FP64 twiddles come from a table tw[m] = exp(-2 pi i m / N) generated in
// extended precision on the host and rounded once.  FP32 transforms (TWC)
// evaluate theirs in registers with the hardware sine and cosine of the angle
// in revolutions (m / N, exact in FP32): no table reads in the passes, at a
// measured 1.3-1.4x the table's rounding error for one 512-point 3D transform
// or right-hand side and the same error after 20 RK4 steps.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pst {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T> __device__ __forceinline__ cx<T> czero() { return {T(0), T(0)}; }
// multiply by i
template <typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
// multiply by exp(-+ i pi / 2): -i for the forward transform, +i for the inverse
template <bool INV, typename T> __device__ __forceinline__ cx<T> rot90(cx<T> a) {
    return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------- butterflies
template <bool INV, typename T> __device__ __forceinline__ void dft2(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV, typename T> __device__ __forceinline__ void dft3(cx<T>* v) {
    const T h = T(0.86602540378443864676);  // sin(2 pi / 3)
    cx<T> s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    cx<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    cx<T> r = cscale(rot90<INV>(d), h);
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

// 4-point DFT of (c0, c1, c2, c3) with stride ST in v
template <bool INV, int ST = 1, typename T> __device__ __forceinline__ void dft4s(cx<T>* v) {
    cx<T> t0 = cadd(v[0], v[2 * ST]), t1 = csub(v[0], v[2 * ST]);
    cx<T> t2 = cadd(v[ST], v[3 * ST]), t3 = rot90<INV>(csub(v[ST], v[3 * ST]));
    v[0] = cadd(t0, t2);
    v[2 * ST] = csub(t0, t2);
    v[ST] = cadd(t1, t3);
    v[3 * ST] = csub(t1, t3);
}
template <bool INV, typename T> __device__ __forceinline__ void dft4(cx<T>* v) { dft4s<INV, 1>(v); }

// multiply by exp(-+ 2 pi i m / 8)
template <bool INV, int M, typename T> __device__ __forceinline__ cx<T> w8(cx<T> a) {
    const T c = T(0.70710678118654752440);
    if constexpr (M == 0) return a;
    else if constexpr (M == 1) return INV ? cx<T>{c * (a.x - a.y), c * (a.x + a.y)} : cx<T>{c * (a.x + a.y), c * (a.y - a.x)};
    else if constexpr (M == 2) return rot90<INV>(a);
    else return INV ? cx<T>{-c * (a.x + a.y), c * (a.x - a.y)} : cx<T>{c * (a.y - a.x), -c * (a.x + a.y)};
}

// 8-point DFT: radix-2 split, twiddle by w8^r, two 4-point DFTs.
template <bool INV, typename T> __device__ __forceinline__ void dft8(cx<T>* v) {
    cx<T> b0 = cadd(v[0], v[4]), b1 = cadd(v[1], v[5]), b2 = cadd(v[2], v[6]), b3 = cadd(v[3], v[7]);
    cx<T> b4 = csub(v[0], v[4]), b5 = w8<INV, 1>(csub(v[1], v[5]));
    cx<T> b6 = w8<INV, 2>(csub(v[2], v[6])), b7 = w8<INV, 3>(csub(v[3], v[7]));
    cx<T> e[4] = {b0, b1, b2, b3}, o[4] = {b4, b5, b6, b7};
    dft4<INV>(e);
    dft4<INV>(o);
    v[0] = e[0]; v[2] = e[1]; v[4] = e[2]; v[6] = e[3];
    v[1] = o[0]; v[3] = o[1]; v[5] = o[2]; v[7] = o[3];
}

// multiply by exp(-+ 2 pi i m / 16)
template <bool INV, int M, typename T> __device__ __forceinline__ cx<T> w16(cx<T> a) {
    if constexpr (M % 2 == 0) return w8<INV, (M / 2) % 8>(a);
    else {
        constexpr double ang = 2.0 * 3.14159265358979323846 * M / 16.0;
        // cos / sin of odd multiples of pi/8, written out
        constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
        constexpr double cs = (M == 1) ? c1 : (M == 3) ? s1 : (M == 5) ? -s1 : (M == 7) ? -c1 : (M == 9) ? -c1 : 0.0;
        constexpr double sn = (M == 1) ? s1 : (M == 3) ? c1 : (M == 5) ? c1 : (M == 7) ? s1 : (M == 9) ? -s1 : 0.0;
        (void)ang;
        const T c = T(cs), s = INV ? T(sn) : T(-sn);
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

// 16-point DFT as 4 x 4: index n = 4 n1 + n2, k = k1 + 4 k2.
template <bool INV, typename T> __device__ __forceinline__ void dft16(cx<T>* v) {
    // first: 4-point DFTs over n1 for each n2 (stride 4)
    dft4s<INV, 4>(v + 0);
    dft4s<INV, 4>(v + 1);
    dft4s<INV, 4>(v + 2);
    dft4s<INV, 4>(v + 3);
    // now v[4 k1 + n2] = Y_{n2}[k1]; twiddle by w16^{n2 k1}
    v[5] = w16<INV, 1>(v[5]);   v[6] = w16<INV, 2>(v[6]);   v[7] = w16<INV, 3>(v[7]);
    v[9] = w16<INV, 2>(v[9]);   v[10] = w16<INV, 4>(v[10]); v[11] = w16<INV, 6>(v[11]);
    v[13] = w16<INV, 3>(v[13]); v[14] = w16<INV, 6>(v[14]); v[15] = w16<INV, 9>(v[15]);
    // second: 4-point DFTs over n2 for each k1 (contiguous groups of 4)
    dft4s<INV, 1>(v + 0);
    dft4s<INV, 1>(v + 4);
    dft4s<INV, 1>(v + 8);
    dft4s<INV, 1>(v + 12);
    // v[4 k1 + k2] = X[k1 + 4 k2]: transpose the 4 x 4 block
    cx<T> t;
    t = v[1];  v[1] = v[4];   v[4] = t;
    t = v[2];  v[2] = v[8];   v[8] = t;
    t = v[3];  v[3] = v[12];  v[12] = t;
    t = v[6];  v[6] = v[9];   v[9] = t;
    t = v[7];  v[7] = v[13];  v[13] = t;
    t = v[11]; v[11] = v[14]; v[14] = t;
}

template <int R, bool INV, typename T> __device__ __forceinline__ void dft(cx<T>* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 16) dft16<INV>(v);
    else static_assert(R == 2, "unsupported radix");
}

// ------------------------------------------------------------ radix schedules
template <int... Rs>
struct Radices {
    static constexpr int S = sizeof...(Rs);
    static constexpr int N = (Rs * ... * 1);
    static constexpr int r[S] = {Rs...};
};

template <class P, bool REV>
__host__ __device__ constexpr int radix_at(int s) { return REV ? P::r[P::S - 1 - s] : P::r[s]; }
template <class P, bool REV>
__host__ __device__ constexpr int span_at(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix_at<P, REV>(i);
    return p;
}

// LDS views.  A line view places one line contiguously with one pad slot
// every 8 points (breaks the power-of-two bank strides of the stage writes);
// a tile view interleaves TL lines, point p of the thread's line at p * TLP.
//
// at(base, delta) is operator()(base + delta) for the case where base + delta
// carries nothing into bit 3 beyond what delta does: delta a multiple of 8, or
// base % 8 + delta < 8.  The padded index then splits into a per-thread part
// and a compile-time offset, so unrolled stages address LDS by immediates.
template <typename T>
struct LineLds {
    cx<T>* p;
    __device__ __forceinline__ cx<T>& operator()(int i) const { return p[i + (i >> 3)]; }
    __device__ __forceinline__ cx<T>& at(int base, int delta) const {
        return p[(base + (base >> 3)) + (delta + (delta >> 3))];
    }
    static constexpr int size(int n) { return n + n / 8; }
};
template <typename T, int TLP>
struct TileLds {
    cx<T>* p;  // already offset by the thread's line
    __device__ __forceinline__ cx<T>& operator()(int i) const { return p[i * TLP]; }
    __device__ __forceinline__ cx<T>& at(int base, int delta) const { return p[(base + delta) * TLP]; }
};
// Block-padded tile view: point i of the TL interleaved lines at
// (i + i / 8) TL, i.e. one empty group of TL slots after every 8 points.  The
// accesses of a radix-8 Stockham stage (points g + r n/R of consecutive g, or
// 8 g + r, or 64 (g / 8) + g % 8 + 8 r) then fall on distinct LDS banks for
// tiles of 4 or 8 lines, where a one-slot pad per point (TileLds) gives
// two-way conflicts; and i / 8 splits into a per-thread base plus a
// compile-time offset for all of them, so no extra address arithmetic.
template <typename T, int TL>
struct TileBlk {
    cx<T>* p;  // already offset by the thread's line
    __device__ __forceinline__ cx<T>& operator()(int i) const { return p[(i + (i >> 3)) * TL]; }
    __device__ __forceinline__ cx<T>& at(int base, int delta) const {
        return p[(base + (base >> 3)) * TL + (delta + (delta >> 3)) * TL];
    }
    static constexpr int size(int n) { return (n + n / 8) * TL; }
};

// Synchronisation of the LDS exchanges between transform stages: the whole
// workgroup, or (WS) only the wavefront, when the G threads of every line are
// lanes of one wavefront.  LDS operations of one wavefront complete in program
// order, so a wavefront-scope fence that keeps the compiler from moving LDS
// accesses across it is enough there.
template <bool WS>
__device__ __forceinline__ void lds_sync() {
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One n-point transform of one line; the caller has loaded v[e] = x[first_pos(g, e)]
// and receives v[e] = X[last_pos(g, e)].  Every thread of the block (WS: of the
// wavefront) must call it: it synchronises between stages with lds_sync<WS>.
// TWC (FP32 only): twiddle factors evaluated in registers by the hardware
// sine / cosine of the angle in revolutions instead of read from the table.
template <typename T, class P, int G, bool INV, bool REV = false, bool WS = false, bool TWC = false>
struct Fft {
    static_assert(!TWC || sizeof(T) == 4, "computed twiddles are FP32 only");
    static constexpr int N = P::N;
    static constexpr int S = P::S;
    static constexpr int E = N / G;
    static constexpr int R_FIRST = radix_at<P, REV>(0);
    static constexpr int R_LAST = radix_at<P, REV>(S - 1);
    static_assert(N % G == 0, "threads per line must divide n");
    static_assert(!WS || 64 % G == 0, "wavefront sync needs the lines inside wavefronts");

    __device__ __forceinline__ static int first_pos(int g, int e) {
        return g + (e / R_FIRST) * G + (e % R_FIRST) * (N / R_FIRST);
    }
    __device__ __forceinline__ static int last_pos(int g, int e) {
        return g + (e / R_LAST) * G + (e % R_LAST) * (N / R_LAST);
    }

    static constexpr int EXCH = S - 1;   // LDS exchanges per transform

    template <int s, bool PP, class Lds>
    __device__ __forceinline__ static void stage(cx<T> (&v)[E], int g, const Lds& l0, const Lds& l1, int ex,
                                                 const cx<T>* __restrict__ tw) {
        constexpr int R = radix_at<P, REV>(s);
        constexpr int NS = span_at<P, REV>(s);
        constexpr int NB = E / R;
        static_assert(E % R == 0, "each thread must own whole butterflies");
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int b = g + i * G;
            if constexpr (s > 0) {
                const int j = b % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> w;
                    if constexpr (TWC) {
                        const float a = (float)(j * r * (N / (NS * R))) * (1.0f / (float)N);
                        w = {__builtin_amdgcn_cosf(a), -__builtin_amdgcn_sinf(a)};
                    } else {
                        w = tw[j * r * (N / (NS * R))];
                    }
                    if (INV) w.y = -w.y;
                    v[i * R + r] = cmul(v[i * R + r], w);
                }
            }
            dft<R, INV>(&v[i * R]);
        }
        if constexpr (s + 1 < S) {
            const Lds lds = (PP && ((ex + s) & 1)) ? l1 : l0;
            constexpr int R2 = radix_at<P, REV>(s + 1);
            constexpr int NB2 = E / R2;
            // writes base + r NS: carry-free when NS is a multiple of 8, or
            // NS R = 8 (then base % 8 = b % NS and base % 8 + r NS < 8);
            // reads g + i G + r N / R2: when G and N / R2 are multiples of 8
            constexpr bool WOK = NS % 8 == 0 || NS * R == 8;
            constexpr bool ROK = G % 8 == 0 && (N / R2) % 8 == 0;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = g + i * G;
                const int base = (b / NS) * NS * R + (b % NS);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (WOK) lds.at(base, r * NS) = v[i * R + r];
                    else lds(base + r * NS) = v[i * R + r];
                }
            }
            lds_sync<WS>();
#pragma unroll
            for (int i = 0; i < NB2; ++i)
#pragma unroll
                for (int r = 0; r < R2; ++r) {
                    if constexpr (ROK) v[i * R2 + r] = lds.at(g, i * G + r * (N / R2));
                    else v[i * R2 + r] = lds(g + i * G + r * (N / R2));
                }
            if constexpr (!PP) lds_sync<WS>();
            stage<s + 1, PP>(v, g, l0, l1, ex, tw);
        }
    }

    template <class Lds>
    __device__ __forceinline__ static void run(cx<T> (&v)[E], int g, const Lds& lds, const cx<T>* __restrict__ tw) {
        stage<0, false>(v, g, lds, lds, 0, tw);
    }

    // Ping-pong form: exchange x of this transform goes through view
    // (ex + x) & 1 of two disjoint LDS buffers, with one barrier between its
    // writes and its reads and none after them.  This is safe when the
    // caller's LDS phases (each: writes, one barrier, reads) strictly alternate
    // between the two buffers: a buffer is rewritten only after the barrier of
    // the phase in between, which every reader of its old contents has passed.
    // The caller continues with phase number ex + EXCH.
    template <class Lds>
    __device__ __forceinline__ static void run_pp(cx<T> (&v)[E], int g, const Lds& l0, const Lds& l1, int ex,
                                                  const cx<T>* __restrict__ tw) {
        stage<0, true>(v, g, l0, l1, ex, tw);
    }
};

}  // namespace pst
