// blas.hip - FP64 vector kernels of the outer flexible GMRES: the classical Gram-Schmidt
// passes (dot products against the Krylov basis and the matching corrections, fused so
// each pass streams w and the basis once), deterministic reductions of the partial sums,
// and the solution update x += Z y.
//
// In the block-tiled FP64 layout every 16-byte vector is one complex component (real
// and imaginary part adjacent) and all FP64 spinor fields share one element order, so
// these kernels treat a vector as a flat array of 12 V complex numbers. FP32 fields
// hold two complex components per 16-byte vector (see zupdate).
//
// Reductions are two-level and in a fixed order: every workgroup writes its partial sum,
// and a second kernel adds the partial sums in workgroup order, so a result never
// depends on which other right-hand sides share the launch.
#include "kernels.hpp"

namespace sapdd {

constexpr int BLAS_WG = 256;

// Basis and Z vectors are streamed once per pass, far beyond the caches: loads carry the
// non-temporal hint (measured 5% faster Gram-Schmidt passes on 32^3x64 with 12 RHS).
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 ldb(const double2 *p) {
    const dv2 v = __builtin_nontemporal_load(reinterpret_cast<const dv2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ldb(const float4 *p) {
    const fv4 v = __builtin_nontemporal_load(reinterpret_cast<const fv4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// The workgroup count (and so the summation order) depends on the vector length only,
// never on how many right-hand sides share the launch.
int blas_partials(int64_t n, int nact) {
    (void)nact;
    int64_t want = (n + 4 * BLAS_WG - 1) / (4 * BLAS_WG);  // about four entries per thread
    const int cap = 1024;  // 4096 measured slower
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    return (int)want;
}

// Partial sums are stored value-major per slot: value k of workgroup q at out[k * nwg]
// relative to the slot's and workgroup's base, so that the reduction of one value reads
// contiguous memory.
template <int NVAL>
__device__ __forceinline__ void wg_reduce_store(double (&v)[NVAL], double *out, int nwg) {
    __shared__ double red[BLAS_WG / 64][NVAL > 0 ? NVAL : 1];
#pragma unroll
    for (int k = 0; k < NVAL; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NVAL; ++k) red[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if ((int)threadIdx.x < NVAL) {
        double t = 0;
#pragma unroll
        for (int q = 0; q < BLAS_WG / 64; ++q) t += red[q][threadIdx.x];
        out[(int64_t)threadIdx.x * nwg] = t;
    }
}

template <int MODE, int NV>
__global__ __launch_bounds__(BLAS_WG) void cgs_kernel(CgsArgs a) {
    constexpr int NVAL = MODE == 2 ? 1 : MODE == 1 ? 2 * NV + 1 : 2 * NV;
    const int slot = blockIdx.y;
    const int rhs = a.active[slot];
    if constexpr (MODE == 2 && NV > 0) {
        // the second correction of classical Gram-Schmidt twice, where it is negligible:
        // w keeps the first pass's result and its norm (the same test on every thread,
        // so the whole workgroup leaves together)
        if (a.skip_tol > 0) {
            const double *c = a.coef + (int64_t)rhs * a.cstride;
            double cc = 0;
#pragma unroll
            for (int i = 0; i < NV; ++i) cc += c[2 * (a.v0 + i)] * c[2 * (a.v0 + i)] + c[2 * (a.v0 + i) + 1] * c[2 * (a.v0 + i) + 1];
            const double wn = c[2 * (a.v0 + NV)];
            if (cc <= a.skip_tol * wn) {
                if (threadIdx.x == 0) a.part[(int64_t)slot * gridDim.x + blockIdx.x] = blockIdx.x == 0 ? wn : 0.0;
                return;
            }
        }
    }
    const double2 *v = (const double2 *)(a.vbase + rhs * a.rstride + (int64_t)a.v0 * a.vstride);
    const int64_t vs = a.vstride / 2;
    double2 *w = (double2 *)(a.w + rhs * a.wstride);
    double cr[NV > 0 ? NV : 1], ci[NV > 0 ? NV : 1];
    if (MODE >= 1) {
        const double *c = a.coef + (int64_t)rhs * a.cstride;
        const double *sc = a.vscale + (int64_t)rhs * a.vsstride;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double s = sc[a.v0 + i];
            cr[i] = c[2 * (a.v0 + i)] * s;
            ci[i] = c[2 * (a.v0 + i) + 1] * s;
        }
    }
    double acc[NVAL];
#pragma unroll
    for (int k = 0; k < NVAL; ++k) acc[k] = 0;
    const int64_t stride = (int64_t)gridDim.x * BLAS_WG;
    for (int64_t e = (int64_t)blockIdx.x * BLAS_WG + threadIdx.x; e < a.n; e += stride) {
        double2 vv[NV > 0 ? NV : 1];
#pragma unroll
        for (int i = 0; i < NV; ++i) vv[i] = ldb(v + i * vs + e);
        double2 ww = w[e];
        if (MODE >= 1 && NV > 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                ww.x -= cr[i] * vv[i].x - ci[i] * vv[i].y;
                ww.y -= cr[i] * vv[i].y + ci[i] * vv[i].x;
            }
            w[e] = ww;
        }
        if (MODE <= 1) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {  // conj(v) w
                acc[2 * i] += vv[i].x * ww.x + vv[i].y * ww.y;
                acc[2 * i + 1] += vv[i].x * ww.y - vv[i].y * ww.x;
            }
            if (MODE == 1) acc[NVAL - 1] += ww.x * ww.x + ww.y * ww.y;
        } else {
            acc[0] += ww.x * ww.x + ww.y * ww.y;
        }
    }
    wg_reduce_store<NVAL>(acc, a.part + (int64_t)slot * NVAL * gridDim.x + blockIdx.x, (int)gridDim.x);
}

template <int MODE, int NV>
static hipError_t cgs_launch(const CgsArgs &a, hipStream_t st) {
    const int nwg = blas_partials(a.n, a.nact);
    hipLaunchKernelGGL((cgs_kernel<MODE, NV>), dim3(nwg, a.nact), dim3(BLAS_WG), 0, st, a);
    return hipGetLastError();
}

template <int MODE>
static hipError_t cgs_mode(const CgsArgs &a, hipStream_t st) {
    if (MODE == 2 && a.nv == 0) return cgs_launch<2, 0>(a, st);  // plain |w|^2
    switch (a.nv) {
#define C(N) case N: return cgs_launch<MODE, N>(a, st);
        C(1) C(2) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16)
#undef C
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cgs(int mode, const CgsArgs &a, hipStream_t st) {
    if (a.nact <= 0) return hipSuccess;
    if (mode == 0) return cgs_mode<0>(a, st);
    if (mode == 1) return cgs_mode<1>(a, st);
    if (mode == 2) return cgs_mode<2>(a, st);
    return hipErrorInvalidValue;
}

// One workgroup per (slot, value): out[rhs * ostride + k] = sum over the nwg partial sums
// of value k, added in a fixed order (times mul[rhs * mstride + v0 + k / 2] if given,
// except for the last value of an odd count);
// for k = 0 also isq[rhs * istride] = 1 / sqrt(sum) if isq is given.
__global__ __launch_bounds__(BLAS_WG) void reduce_kernel(const double *part, int nwg, int nval, const int *active,
                                                         double *out, int ostride, const double *mul, int mstride,
                                                         int v0, double *isq, int istride) {
    __shared__ double red[BLAS_WG / 64];
    const int slot = blockIdx.x;
    const int k = blockIdx.y;
    const int rhs = active[slot];
    const double *p = part + ((int64_t)slot * nval + k) * nwg;
    double t = 0;
    for (int q = threadIdx.x; q < nwg; q += BLAS_WG) t += p[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int q = 0; q < BLAS_WG / 64; ++q) s += red[q];
        if (mul && k < (nval & ~1)) s *= mul[(int64_t)rhs * mstride + v0 + k / 2];
        out[(int64_t)rhs * ostride + k] = s;
        if (isq && k == 0) isq[(int64_t)rhs * istride] = s > 0 ? 1.0 / sqrt(s) : 0.0;
    }
}

hipError_t launch_reduce(const double *part, int nwg, int nval, const int *active, int nact, double *out,
                         int ostride, const double *mul, int mstride, int v0, double *isq, int istride,
                         hipStream_t st) {
    if (nact <= 0 || nval <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(nact, nval), dim3(BLAS_WG), 0, st, part, nwg, nval, active, out, ostride,
                       mul, mstride, v0, isq, istride);
    return hipGetLastError();
}

// In place, for every listed slot: v_l <- sum_{i < NIN} s_i v_i P_il for l < nout (FP64
// complex vectors of n entries), with s_i = vscale[rhs * vsstride + i] (1 without
// vscale) and P column-major with leading dimension ld at P + rhs * pstride (complex).
// Each thread holds all NIN entries of its element before writing any, so outputs may
// overwrite inputs.
template <int NIN>
__global__ __launch_bounds__(BLAS_WG) void recombine_kernel(double *base, int64_t rstride, int64_t vstride,
                                                            const double *vscale, int vsstride, const double *P,
                                                            int64_t pstride, int ld, int nout, const int *active,
                                                            int64_t n) {
    const int rhs = active[blockIdx.y];
    double2 *b = (double2 *)(base + rhs * rstride);
    const int64_t vs = vstride / 2;
    const double *pm = P + rhs * pstride;
    double sc[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) sc[i] = vscale ? vscale[(int64_t)rhs * vsstride + i] : 1.0;
    const int64_t stride = (int64_t)gridDim.x * BLAS_WG;
    for (int64_t e = (int64_t)blockIdx.x * BLAS_WG + threadIdx.x; e < n; e += stride) {
        double2 v[NIN];
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            v[i] = b[i * vs + e];
            v[i].x *= sc[i];
            v[i].y *= sc[i];
        }
        for (int l = 0; l < nout; ++l) {
            double re = 0, im = 0;
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
                const double pr = pm[2 * (i + ld * l)], pi = pm[2 * (i + ld * l) + 1];
                re = __builtin_fma(v[i].x, pr, __builtin_fma(-v[i].y, pi, re));
                im = __builtin_fma(v[i].x, pi, __builtin_fma(v[i].y, pr, im));
            }
            b[l * vs + e] = make_double2(re, im);
        }
    }
}

__global__ void set_scales_kernel(double *vscale, int vsstride, int count, const int *active) {
    const int rhs = active[blockIdx.x];
    if ((int)threadIdx.x < count) vscale[(int64_t)rhs * vsstride + threadIdx.x] = 1.0;
}

hipError_t launch_recombine(double *base, int64_t rstride, int64_t vstride, const double *vscale, int vsstride,
                            const double *P, int64_t pstride, int ld, int nin, int nout, const int *active, int nact,
                            int64_t n, hipStream_t st) {
    if (nact <= 0 || nout <= 0) return hipSuccess;
    if (nout > nin) return hipErrorInvalidValue;
    const dim3 grid(blas_partials(n, nact), nact);
    switch (nin) {
#define C(N)                                                                                                     \
    case N:                                                                                                      \
        hipLaunchKernelGGL(recombine_kernel<N>, grid, dim3(BLAS_WG), 0, st, base, rstride, vstride, vscale,      \
                           vsstride, P, pstride, ld, nout, active, n);                                            \
        break;
        C(1) C(2) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16) C(17)
#undef C
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !vscale) return e;
    hipLaunchKernelGGL(set_scales_kernel, dim3(nact), dim3(64), 0, st, (double *)vscale, vsstride, nout, active);
    return hipGetLastError();
}

// x += sum_j y_j z_j. FP64 z shares x's element order; an FP32 z holds the complex
// components 2v and 2v + 1 of site (bp, s) in its float4 number (bp * 6 + v) * Vbh + s,
// which map to the double2 numbers (bp * 12 + 2v) * Vbh + s and the one Vbh later.
__global__ __launch_bounds__(BLAS_WG) void zupdate64_kernel(double *x, int64_t xstride, const double *z, int64_t zsj,
                                                            int64_t zsr, const double *y, int ystride, int nz,
                                                            const int *active, int64_t n) {
    const int rhs = active[blockIdx.y];
    double2 *xr = (double2 *)(x + rhs * xstride);
    const double2 *zr = (const double2 *)(z + rhs * zsr);
    const double *yr = y + (int64_t)rhs * ystride;
    const int64_t stride = (int64_t)gridDim.x * BLAS_WG;
    for (int64_t e = (int64_t)blockIdx.x * BLAS_WG + threadIdx.x; e < n; e += stride) {
        double2 acc = xr[e];
        for (int j = 0; j < nz; ++j) {
            const double2 q = ldb(zr + j * (zsj / 2) + e);
            acc.x += yr[2 * j] * q.x - yr[2 * j + 1] * q.y;
            acc.y += yr[2 * j] * q.y + yr[2 * j + 1] * q.x;
        }
        xr[e] = acc;
    }
}

__global__ __launch_bounds__(BLAS_WG) void zupdate32_kernel(double *x, int64_t xstride, const float *z, int64_t zsj,
                                                            int64_t zsr, const double *y, int ystride, int nz,
                                                            const int *active, int64_t n4, int vbh) {
    const int rhs = active[blockIdx.y];
    double2 *xr = (double2 *)(x + rhs * xstride);
    const float4 *zr = (const float4 *)(z + rhs * zsr);
    const double *yr = y + (int64_t)rhs * ystride;
    const int64_t stride = (int64_t)gridDim.x * BLAS_WG;
    for (int64_t q = (int64_t)blockIdx.x * BLAS_WG + threadIdx.x; q < n4; q += stride) {
        const int64_t t = q / vbh;
        const int s = (int)(q - t * vbh);
        const int64_t e0 = (2 * t) * vbh + s;  // (bp * 12 + 2v) * Vbh + s with t = bp * 6 + v
        double2 a0 = xr[e0], a1 = xr[e0 + vbh];
        for (int j = 0; j < nz; ++j) {
            const float4 f = ldb(zr + j * (zsj / 4) + q);
            const double yr_ = yr[2 * j], yi_ = yr[2 * j + 1];
            a0.x += yr_ * f.x - yi_ * f.y;
            a0.y += yr_ * f.y + yi_ * f.x;
            a1.x += yr_ * f.z - yi_ * f.w;
            a1.y += yr_ * f.w + yi_ * f.z;
        }
        xr[e0] = a0;
        xr[e0 + vbh] = a1;
    }
}

hipError_t launch_zupdate(double *x, int64_t xstride, const void *z, int zprec, int64_t zstride_j,
                          int64_t zstride_rhs, const double *y, int ystride, int nz, const int *active, int nact,
                          int64_t n, int vbh, hipStream_t st) {
    if (nact <= 0 || nz <= 0) return hipSuccess;
    const int nwg = blas_partials(n, nact);
    if (zprec == P64)
        hipLaunchKernelGGL(zupdate64_kernel, dim3(nwg, nact), dim3(BLAS_WG), 0, st, x, xstride, (const double *)z,
                           zstride_j, zstride_rhs, y, ystride, nz, active, n);
    else if (zprec == P32)
        hipLaunchKernelGGL(zupdate32_kernel, dim3(nwg, nact), dim3(BLAS_WG), 0, st, x, xstride, (const float *)z,
                           zstride_j, zstride_rhs, y, ystride, nz, active, n / 2, vbh);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace sapdd
