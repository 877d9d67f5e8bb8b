// layout.hip - conversions between the canonical site-major FP64 arrays and the
// block-tiled even-odd SoA layout (FP64, FP32 or FP16 with a per-site FP32 scale), and
// a STREAM-type copy kernel used to measure attainable HBM bandwidth.
#include "core.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace sapdd {

constexpr int LAYOUT_WG = 256;

// Canonical site index (x fastest) of block-tiled site (bp, s).
__device__ __forceinline__ int64_t canon_index(const Geom &geo, int64_t bp, int s) {
    int x[4];
    coords_of(geo, bp, s, x);
    return x[0] + (int64_t)geo.L[0] * (x[1] + (int64_t)geo.L[1] * (x[2] + (int64_t)geo.L[2] * x[3]));
}

template <int N, class S>
__global__ __launch_bounds__(LAYOUT_WG) void pack_kernel(Geom geo, const double *__restrict__ canon, S *out,
                                                         float *scale) {
    const int64_t t = (int64_t)blockIdx.x * LAYOUT_WG + threadIdx.x;
    if (t >= geo.V) return;
    const int f = blockIdx.y;
    const int64_t bp = t / geo.Vbh;
    const int s = (int)(t - bp * geo.Vbh);
    const double *src = canon + ((int64_t)f * geo.V + canon_index(geo, bp, s)) * N;
    double v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = src[k];
    store_site<double, N>(out + (int64_t)f * geo.V * N, scale ? scale + (int64_t)f * geo.V : nullptr, bp, s, geo.Vbh,
                          v);
}

template <int N, class S>
__global__ __launch_bounds__(LAYOUT_WG) void unpack_kernel(Geom geo, const S *in, const float *scale,
                                                           double *__restrict__ canon) {
    const int64_t t = (int64_t)blockIdx.x * LAYOUT_WG + threadIdx.x;
    if (t >= geo.V) return;
    const int f = blockIdx.y;
    const int64_t bp = t / geo.Vbh;
    const int s = (int)(t - bp * geo.Vbh);
    double v[N];
    load_site<double, N>(in + (int64_t)f * geo.V * N, scale ? scale + (int64_t)f * geo.V : nullptr, bp, s, geo.Vbh, v);
    double *dst = canon + ((int64_t)f * geo.V + canon_index(geo, bp, s)) * N;
#pragma unroll
    for (int k = 0; k < N; ++k) dst[k] = v[k];
}

template <int N, class S>
__global__ __launch_bounds__(LAYOUT_WG) void convert_kernel(Geom geo, const double *__restrict__ in, S *out,
                                                            float *scale) {
    const int64_t t = (int64_t)blockIdx.x * LAYOUT_WG + threadIdx.x;
    if (t >= geo.V) return;
    const int f = blockIdx.y;
    const int64_t bp = t / geo.Vbh;
    const int s = (int)(t - bp * geo.Vbh);
    double v[N];
    load_site<double, N>(in + (int64_t)f * geo.V * N, nullptr, bp, s, geo.Vbh, v);
    store_site<double, N>(out + (int64_t)f * geo.V * N, scale ? scale + (int64_t)f * geo.V : nullptr, bp, s, geo.Vbh,
                          v);
}

static dim3 site_grid(const Geom &geo, int nfield) {
    return dim3((unsigned)((geo.V + LAYOUT_WG - 1) / LAYOUT_WG), (unsigned)nfield);
}

template <int N>
static hipError_t pack_n(const Geom &geo, int nfield, const double *canon, Fld out, hipStream_t st) {
    const dim3 g = site_grid(geo, nfield);
    if (out.prec == P64) hipLaunchKernelGGL((pack_kernel<N, double>), g, dim3(LAYOUT_WG), 0, st, geo, canon, (double *)out.data, nullptr);
    else if (out.prec == P32) hipLaunchKernelGGL((pack_kernel<N, float>), g, dim3(LAYOUT_WG), 0, st, geo, canon, (float *)out.data, nullptr);
    else hipLaunchKernelGGL((pack_kernel<N, half_t>), g, dim3(LAYOUT_WG), 0, st, geo, canon, (half_t *)out.data, out.scale);
    return hipGetLastError();
}

template <int N>
static hipError_t unpack_n(const Geom &geo, int nfield, Fld in, double *canon, hipStream_t st) {
    const dim3 g = site_grid(geo, nfield);
    if (in.prec == P64) hipLaunchKernelGGL((unpack_kernel<N, double>), g, dim3(LAYOUT_WG), 0, st, geo, (const double *)in.data, nullptr, canon);
    else if (in.prec == P32) hipLaunchKernelGGL((unpack_kernel<N, float>), g, dim3(LAYOUT_WG), 0, st, geo, (const float *)in.data, nullptr, canon);
    else hipLaunchKernelGGL((unpack_kernel<N, half_t>), g, dim3(LAYOUT_WG), 0, st, geo, (const half_t *)in.data, in.scale, canon);
    return hipGetLastError();
}

template <int N>
static hipError_t convert_n(const Geom &geo, int nfield, const double *in, Fld out, hipStream_t st) {
    const dim3 g = site_grid(geo, nfield);
    if (out.prec == P64) return hipErrorInvalidValue;
    if (out.prec == P32) hipLaunchKernelGGL((convert_kernel<N, float>), g, dim3(LAYOUT_WG), 0, st, geo, in, (float *)out.data, nullptr);
    else hipLaunchKernelGGL((convert_kernel<N, half_t>), g, dim3(LAYOUT_WG), 0, st, geo, in, (half_t *)out.data, out.scale);
    return hipGetLastError();
}

hipError_t launch_pack(const Geom &geo, int ncomp, int nfield, const double *canon, Fld out, hipStream_t st) {
    if (nfield <= 0 || geo.V == 0) return hipSuccess;
    if (ncomp == 24) return pack_n<24>(geo, nfield, canon, out, st);
    if (ncomp == 72) return pack_n<72>(geo, nfield, canon, out, st);
    return hipErrorInvalidValue;
}

hipError_t launch_unpack(const Geom &geo, int ncomp, int nfield, Fld in, double *canon, hipStream_t st) {
    if (nfield <= 0 || geo.V == 0) return hipSuccess;
    if (ncomp == 24) return unpack_n<24>(geo, nfield, in, canon, st);
    if (ncomp == 72) return unpack_n<72>(geo, nfield, in, canon, st);
    return hipErrorInvalidValue;
}

hipError_t launch_convert(const Geom &geo, int ncomp, int nfield, const double *in, Fld out, hipStream_t st) {
    if (nfield <= 0 || geo.V == 0) return hipSuccess;
    if (ncomp == 24) return convert_n<24>(geo, nfield, in, out, st);
    if (ncomp == 72) return convert_n<72>(geo, nfield, in, out, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- copy (bandwidth probe)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte vector per thread over a grid that covers the whole buffer, with
// non-temporal hints: measured 6.2-6.5 TB/s on 2 GiB, where a grid capped at 16k
// workgroups that strides over the buffer stayed at 4.4-5.3 TB/s.
__global__ __launch_bounds__(256) void copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, int64_t n16,
                                                   int64_t base, const unsigned char *__restrict__ tsrc,
                                                   unsigned char *__restrict__ tdst, int tail) {
    const int64_t i = base + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    if (base == 0 && blockIdx.x == 0 && (int)threadIdx.x < tail) tdst[threadIdx.x] = tsrc[threadIdx.x];
}

hipError_t launch_copy(const void *src, void *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t n16 = n / 16;
    const int tail = (int)(n - n16 * 16);
    const int64_t per = (int64_t)0x40000000;  // vectors per launch (2^22 workgroups of 256)
    for (int64_t base = 0; base == 0 || base < n16; base += per) {
        int64_t nb = (std::min(per, n16 - base) + 255) / 256;
        if (nb < 1) nb = 1;
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)nb), dim3(256), 0, st, (const u32x4 *)src, (u32x4 *)dst, n16,
                           base, (const unsigned char *)src + n16 * 16, (unsigned char *)dst + n16 * 16, tail);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sapdd
