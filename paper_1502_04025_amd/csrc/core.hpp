// core.hpp - device-side building blocks shared by the sapdd kernels.
//
// * Block-tiled even-odd layout, structure of short arrays (the GPU re-make of the SoA
//   layout of Sec. 3.2): the reals of a site are grouped into 16-byte vectors of W reals
//   (W = 2 doubles, 4 floats or 8 halves); for a field with N reals per site, vector v of
//   the site with parity p and half-site index s in Schwarz block b is vector number
//       ((b * 2 + p) * (N / W) + v) * Vbh + s,      Vbh = (sites per block) / 2.
//   Lane s of a wave loads one whole vector per instruction and a wave reads 1 KB
//   contiguous; the real and imaginary parts of a complex component are adjacent.
//   In FP16 storage every site also carries one FP32 scale at (b * 2 + p) * Vbh + s.
// * Spinor reals: index 2 * (3 * spin + colour) + (0 re, 1 im), 24 per site.
//   Links: 4 directions x 18 reals, index 18 * mu + 2 * (3 * row + col) + re/im.
//   Clover (two chiral 6x6 Hermitian blocks): 36 reals per block, first the 6 real
//   diagonal entries, then the 15 upper off-diagonal entries (i < j, row major) as
//   complex pairs; block k covers spins 2k, 2k+1 and element index 3 * (spin - 2k) + c.
// * DeGrand-Rossi gamma matrices: gamma_mu = [[0, G_mu], [G_mu^+, 0]] with
//   G_x = i sigma_x, G_y = -i sigma_y, G_z = i sigma_z, G_t = 1. Every row of G_mu holds
//   one entry, a power of i, which the projections below apply as add/sub/swap.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sapdd {

typedef _Float16 half_t;

// ------------------------------------------------------------------ storage traits
template <class S> struct Storage;
template <> struct Storage<double> {
    static constexpr bool scaled = false;
    static constexpr int bytes = 8;
};
template <> struct Storage<float> {
    static constexpr bool scaled = false;
    static constexpr int bytes = 4;
};
template <> struct Storage<half_t> {
    static constexpr bool scaled = true;
    static constexpr int bytes = 2;
};

// 16-byte vector of a storage type: the unit one lane loads or stores.
template <class S> struct Vec;
template <> struct Vec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int W = 2;
};
template <> struct Vec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int W = 4;
};
template <> struct Vec<half_t> {
    typedef half_t type __attribute__((ext_vector_type(8)));
    static constexpr int W = 8;
};

// Index (in vectors) of vector v of site (bp, s) in a field of N reals per site.
template <class S, int N>
__host__ __device__ __forceinline__ int64_t vec_index(int64_t bp, int v, int s, int Vbh) {
    static_assert(N % Vec<S>::W == 0, "field width must be a multiple of the vector width");
    return (bp * (N / Vec<S>::W) + v) * (int64_t)Vbh + s;
}
// Index (in reals) of real k of site (bp, s).
template <class S, int N>
__host__ __device__ __forceinline__ int64_t real_index(int64_t bp, int k, int s, int Vbh) {
    return vec_index<S, N>(bp, k / Vec<S>::W, s, Vbh) * Vec<S>::W + k % Vec<S>::W;
}

// A field in the block-tiled layout: data plus (FP16 only) per-site scales.
template <class S> struct FieldPtr {
    S *data;
    float *scale;
};
template <class S> struct CFieldPtr {
    const S *data;
    const float *scale;
};

// Every field these helpers touch lives in device (global) memory. Pointers that pass
// through structs lose that information in the compiler, which then emits flat
// instructions: those also count against the LDS wait counter, so an LDS read would wait
// for every outstanding field load. The casts below keep them global loads and stores.
#define SAPDD_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ const SAPDD_GLOBAL T *gmem(const T *p) { return (const SAPDD_GLOBAL T *)p; }
template <class T> __device__ __forceinline__ SAPDD_GLOBAL T *gmem(T *p) { return (SAPDD_GLOBAL T *)p; }

// One 16-byte vector load / store. NT = true marks data that is streamed through once
// (non-temporal cache hint); fields that other workgroups re-read keep the default.
template <bool NT, class VT> __device__ __forceinline__ VT ld_vec(const VT *p) {
    if constexpr (NT) return __builtin_nontemporal_load(gmem(p));
    else return *gmem(p);
}
template <bool NT, class VT> __device__ __forceinline__ void st_vec(VT *p, const VT &x) {
    if constexpr (NT) __builtin_nontemporal_store(x, gmem(p));
    else *gmem(p) = x;
}

// Reals [K0, K0 + K) of site (bp, s) of an N-real field, through whole 16-byte vectors.
// With RAW the FP16 site scale is not applied (the caller folds it into a result).
template <class R, int N, int K0, int K, class S, bool RAW = false, bool NT = false>
__device__ __forceinline__ void load_reals(const S *__restrict__ data, const float *__restrict__ scale, int64_t bp,
                                           int s, int Vbh, R out[K]) {
    typedef typename Vec<S>::type VT;
    constexpr int W = Vec<S>::W;
    constexpr int v0 = K0 / W, v1 = (K0 + K - 1) / W;
    const VT *p = reinterpret_cast<const VT *>(data);
    R sc = (R)1;
    if constexpr (Storage<S>::scaled && !RAW) sc = (R)*gmem(scale + bp * Vbh + s);
#pragma unroll
    for (int v = v0; v <= v1; ++v) {
        const VT x = ld_vec<NT>(p + vec_index<S, N>(bp, v, s, Vbh));
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int k = v * W + w - K0;
            if (k >= 0 && k < K) {
                if constexpr (Storage<S>::scaled && !RAW) out[k] = (R)(float)x[w] * sc;
                else if constexpr (Storage<S>::scaled) out[k] = (R)(float)x[w];
                else out[k] = (R)x[w];
            }
        }
    }
}

// FP16 per-site scale of site (bp, s) (1 for unscaled storage).
template <class R, class S>
__device__ __forceinline__ R site_scale(const float *__restrict__ scale, int64_t bp, int s, int Vbh) {
    if constexpr (Storage<S>::scaled) return (R)*gmem(scale + bp * Vbh + s);
    else return (R)1;
}

template <class R, int N, class S, bool NT = false>
__device__ __forceinline__ void load_site(const S *__restrict__ data, const float *__restrict__ scale,
                                          int64_t bp, int s, int Vbh, R out[N]) {
    load_reals<R, N, 0, N, S, false, NT>(data, scale, bp, s, Vbh, out);
}

// Reciprocal of an FP16 site scale m (the site's max |value|). A site whose maximum lies
// below the smallest normal float is stored as zero with scale 0: 1/m would overflow to
// +inf there, and 0 * inf = NaN would poison the whole site.
__host__ __device__ __forceinline__ float fp16_site_inv(float m) { return m >= 1.17549435e-38f ? 1.0f / m : 0.f; }

// Store N reals of one site; FP16 storage divides by the site's max |value| and rounds
// to nearest even (scale 0 stores zeros).
template <class R, int N, class S, bool NT = false>
__device__ __forceinline__ void store_site(S *__restrict__ data, float *__restrict__ scale, int64_t bp,
                                           int s, int Vbh, const R in[N]) {
    typedef typename Vec<S>::type VT;
    constexpr int W = Vec<S>::W;
    VT *p = reinterpret_cast<VT *>(data);
    if constexpr (Storage<S>::scaled) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < N; ++k) m = fmaxf(m, fabsf((float)in[k]));
        const float inv = fp16_site_inv(m);
        *gmem(scale + bp * Vbh + s) = inv > 0.f ? m : 0.f;
#pragma unroll
        for (int v = 0; v < N / W; ++v) {
            VT x;
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = (half_t)((float)in[v * W + w] * inv);
            st_vec<NT>(p + vec_index<S, N>(bp, v, s, Vbh), x);
        }
    } else {
#pragma unroll
        for (int v = 0; v < N / W; ++v) {
            VT x;
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = (S)in[v * W + w];
            st_vec<NT>(p + vec_index<S, N>(bp, v, s, Vbh), x);
        }
    }
}

// ------------------------------------------------------------------ arithmetic
// Fused multiply-add in the arithmetic type (one v_fma per call; with an FP16 operand
// converted in place the compiler forms v_fma_mix).
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------------------ gamma structure
// Multiply (re, im) by i^ph.
template <int PH, class R> __device__ __forceinline__ void iph(R re, R im, R &ore, R &oim) {
    if constexpr (PH == 0) { ore = re; oim = im; }
    else if constexpr (PH == 1) { ore = -im; oim = re; }
    else if constexpr (PH == 2) { ore = -re; oim = -im; }
    else { ore = im; oim = -re; }
}

// Row r of G_mu: column and phase exponent (entry = i^phase).
template <int MU, int ROW> struct Grow;
template <> struct Grow<0, 0> { static constexpr int col = 1, ph = 1; };
template <> struct Grow<0, 1> { static constexpr int col = 0, ph = 1; };
template <> struct Grow<1, 0> { static constexpr int col = 1, ph = 2; };
template <> struct Grow<1, 1> { static constexpr int col = 0, ph = 0; };
template <> struct Grow<2, 0> { static constexpr int col = 0, ph = 1; };
template <> struct Grow<2, 1> { static constexpr int col = 1, ph = 3; };
template <> struct Grow<3, 0> { static constexpr int col = 0, ph = 0; };
template <> struct Grow<3, 1> { static constexpr int col = 1, ph = 0; };
// Row r of G_mu^+.
template <int MU, int ROW> struct GDrow;
template <> struct GDrow<0, 0> { static constexpr int col = 1, ph = 3; };
template <> struct GDrow<0, 1> { static constexpr int col = 0, ph = 3; };
template <> struct GDrow<1, 0> { static constexpr int col = 1, ph = 0; };
template <> struct GDrow<1, 1> { static constexpr int col = 0, ph = 2; };
template <> struct GDrow<2, 0> { static constexpr int col = 0, ph = 3; };
template <> struct GDrow<2, 1> { static constexpr int col = 1, ph = 1; };
template <> struct GDrow<3, 0> { static constexpr int col = 0, ph = 0; };
template <> struct GDrow<3, 1> { static constexpr int col = 1, ph = 0; };

// Project a spinor with (1 - SIGN*gamma_mu)... expressed through its upper half:
//   (1 - gamma) psi: h = psi_up - G psi_lo,  lower part = -G^+ h
//   (1 + gamma) psi: h = psi_up + G psi_lo,  lower part = +G^+ h
// SIGN = -1 for (1 - gamma_mu), +1 for (1 + gamma_mu). h has 12 reals (2 spins x 3 colours).
template <int MU, int SIGN, class R>
__device__ __forceinline__ void project(const R psi[24], R h[12]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        {
            constexpr int col = Grow<MU, 0>::col, ph = Grow<MU, 0>::ph;
            R re, im;
            iph<ph>(psi[2 * (3 * (2 + col) + c)], psi[2 * (3 * (2 + col) + c) + 1], re, im);
            h[2 * c] = psi[2 * c] + (R)SIGN * re;
            h[2 * c + 1] = psi[2 * c + 1] + (R)SIGN * im;
        }
        {
            constexpr int col = Grow<MU, 1>::col, ph = Grow<MU, 1>::ph;
            R re, im;
            iph<ph>(psi[2 * (3 * (2 + col) + c)], psi[2 * (3 * (2 + col) + c) + 1], re, im);
            h[2 * (3 + c)] = psi[2 * (3 + c)] + (R)SIGN * re;
            h[2 * (3 + c) + 1] = psi[2 * (3 + c) + 1] + (R)SIGN * im;
        }
    }
}

// acc += scale * reconstruct(h) where reconstruct puts h in the upper spins and
// SIGN * G^+ h in the lower spins.
template <int MU, int SIGN, class R>
__device__ __forceinline__ void accum_recon(R acc[24], const R h[12], R scale) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = fmac(scale, h[k], acc[k]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        {
            constexpr int col = GDrow<MU, 0>::col, ph = GDrow<MU, 0>::ph;
            R re, im;
            iph<ph>(h[2 * (3 * col + c)], h[2 * (3 * col + c) + 1], re, im);
            acc[2 * (6 + c)] = fmac((R)SIGN * scale, re, acc[2 * (6 + c)]);
            acc[2 * (6 + c) + 1] = fmac((R)SIGN * scale, im, acc[2 * (6 + c) + 1]);
        }
        {
            constexpr int col = GDrow<MU, 1>::col, ph = GDrow<MU, 1>::ph;
            R re, im;
            iph<ph>(h[2 * (3 * col + c)], h[2 * (3 * col + c) + 1], re, im);
            acc[2 * (9 + c)] = fmac((R)SIGN * scale, re, acc[2 * (9 + c)]);
            acc[2 * (9 + c) + 1] = fmac((R)SIGN * scale, im, acc[2 * (9 + c) + 1]);
        }
    }
}

// ------------------------------------------------------------------ SU(3) on half spinors
// out = U h for both spins; U has 18 reals, row major complex. Four FMAs per complex
// multiply-add; the first product of each sum is an FMA onto zero as well (its value,
// except that an exact -0 becomes +0), so every term is one fused instruction.
template <class R> __device__ __forceinline__ void su3_mul(const R u[18], const R h[12], R out[12]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R re = fmac(u[2 * (3 * a)], h[2 * (3 * sp)], (R)0);
            R im = fmac(u[2 * (3 * a)], h[2 * (3 * sp) + 1], (R)0);
            re = fmac(-u[2 * (3 * a) + 1], h[2 * (3 * sp) + 1], re);
            im = fmac(u[2 * (3 * a) + 1], h[2 * (3 * sp)], im);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                const R ur = u[2 * (3 * a + b)], ui = u[2 * (3 * a + b) + 1];
                const R hr = h[2 * (3 * sp + b)], hi = h[2 * (3 * sp + b) + 1];
                re = fmac(ur, hr, re);
                re = fmac(-ui, hi, re);
                im = fmac(ur, hi, im);
                im = fmac(ui, hr, im);
            }
            out[2 * (3 * sp + a)] = re;
            out[2 * (3 * sp + a) + 1] = im;
        }
}

// out = U^+ h for both spins.
template <class R> __device__ __forceinline__ void su3_dag_mul(const R u[18], const R h[12], R out[12]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R re = fmac(u[2 * a], h[2 * (3 * sp)], (R)0);
            R im = fmac(u[2 * a], h[2 * (3 * sp) + 1], (R)0);
            re = fmac(u[2 * a + 1], h[2 * (3 * sp) + 1], re);
            im = fmac(-u[2 * a + 1], h[2 * (3 * sp)], im);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                const R ur = u[2 * (3 * b + a)], ui = u[2 * (3 * b + a) + 1];
                const R hr = h[2 * (3 * sp + b)], hi = h[2 * (3 * sp + b) + 1];
                re = fmac(ur, hr, re);
                re = fmac(ui, hi, re);
                im = fmac(ur, hi, im);
                im = fmac(-ui, hr, im);
            }
            out[2 * (3 * sp + a)] = re;
            out[2 * (3 * sp + a) + 1] = im;
        }
}

// ------------------------------------------------------------------ geometry
struct Geom {
    int L[4];  // lattice extents x, y, z, t
    int B[4];  // Schwarz block extents
    int G[4];  // block grid extents L / B
    int Vb, Vbh;
    int64_t Nd, V;
    int antiperiodic;
};

// Local coordinates of half-site s with parity p in a block of extents B.
__host__ __device__ __forceinline__ void local_coords(const int B[4], int p, int s, int l[4]) {
    const int hx = B[0] >> 1;
    int r = s / hx;
    const int xh = s - r * hx;
    l[1] = r % B[1];
    r /= B[1];
    l[2] = r % B[2];
    l[3] = r / B[2];
    const int q = (p + l[1] + l[2] + l[3]) & 1;
    l[0] = 2 * xh + q;
}

__host__ __device__ __forceinline__ int local_half_index(const int B[4], const int l[4]) {
    return (l[0] + B[0] * (l[1] + B[1] * (l[2] + B[2] * l[3]))) >> 1;
}

__host__ __device__ __forceinline__ void block_coords(const int G[4], int64_t b, int g[4]) {
    g[0] = (int)(b % G[0]);
    b /= G[0];
    g[1] = (int)(b % G[1]);
    b /= G[1];
    g[2] = (int)(b % G[2]);
    g[3] = (int)(b / G[2]);
}

__host__ __device__ __forceinline__ int64_t block_index(const int G[4], const int g[4]) {
    return ((int64_t)(g[3] * G[2] + g[2]) * G[1] + g[1]) * G[0] + g[0];
}

// Site address (bp = 2 b + p, s) of global coordinates x[4].
__host__ __device__ __forceinline__ void site_of(const Geom &geo, const int x[4], int64_t &bp, int &s) {
    int g[4], l[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        g[mu] = x[mu] / geo.B[mu];
        l[mu] = x[mu] - g[mu] * geo.B[mu];
    }
    const int p = (l[0] + l[1] + l[2] + l[3]) & 1;
    bp = block_index(geo.G, g) * 2 + p;
    s = local_half_index(geo.B, l);
}

// Global coordinates of site (bp, s).
__host__ __device__ __forceinline__ void coords_of(const Geom &geo, int64_t bp, int s, int x[4]) {
    int g[4], l[4];
    block_coords(geo.G, bp >> 1, g);
    local_coords(geo.B, (int)(bp & 1), s, l);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) x[mu] = g[mu] * geo.B[mu] + l[mu];
}

// b-th block (in colour order) of colour c: blocks of one colour are enumerated row by
// row along x; every x row of the (even-sized) block grid holds G_x / 2 of them.
__host__ __device__ __forceinline__ int64_t colour_block(const int G[4], int c, int64_t k) {
    const int hg = G[0] >> 1;
    const int64_t row = k / hg;
    const int j = (int)(k - row * hg);
    const int gy = (int)(row % G[1]);
    const int64_t r2 = row / G[1];
    const int gz = (int)(r2 % G[2]);
    const int gt = (int)(r2 / G[2]);
    const int gx = 2 * j + ((c + gy + gz + gt) & 1);
    return ((int64_t)(gt * G[2] + gz) * G[1] + gy) * G[0] + gx;
}

}  // namespace sapdd
