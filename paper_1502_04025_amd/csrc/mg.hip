// mg.hip - kernels of the two-level aggregation multigrid preconditioner whose smoother
// is the Schwarz procedure (Sec. 2.6: the group's multigrid solver is a Krylov method
// preconditioned by a multigrid cycle with the domain-decomposition preconditioner of
// Sec. 3.1 as its smoother).
//
// Aggregates are the Schwarz blocks, each split into its two chiralities: spins 0, 1
// and spins 2, 3, the two eigenspaces of gamma_5 in the DeGrand-Rossi basis. The
// interpolation P holds nvec FP32 spinor fields in the block-tiled layout; coarse index
// k = s * nvec + j is the chirality-s half of field j on each aggregate, orthonormal
// per aggregate and chirality. Coarse vectors are complex FP32 arrays [aggregate][K]
// (K = 2 nvec, aggregates in block order, x fastest). The Galerkin operator
// D_c = P^H M P couples an aggregate to itself and its eight neighbours; it is stored
// as nine K x K blocks per aggregate, column-major within a block so that the K rows
// of one column are contiguous: element (row, col) of block d at
// ((b * 9 + d) * K + col) * K + row, d = 0 the aggregate itself, d = 1 + 2 mu the
// forward and d = 2 + 2 mu the backward neighbour in direction mu.
//
// The coarse system is solved by a fixed number of restarted GMRES cycles of a fixed
// number of steps, from zero, entirely on the device so the whole preconditioner is one
// static launch sequence. Classical Gram-Schmidt, in one of two forms chosen when the
// multigrid is set up: every Arnoldi step two kernels (operator + the dot products, then
// correction + norm), which suits batches of systems, or one kernel (correction of the
// previous step's product at the rows it needs, its norm, the operator and the dot
// products of the next), which suits a single system. Each reduction is a fixed-order
// sum of per-workgroup partials that every workgroup of the next kernel repeats for
// itself; one wave per system solves the small
// least squares problem at the end of a cycle, and the cycle's correction is added to
// the coarse solution, whose residual starts the next.
#include "kernels.hpp"

namespace sapdd {

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));

__host__ __device__ __forceinline__ int mg_colour(const int g[4], const MgColouring &cl) {
    return (((g[3] % cl.m[3]) * cl.m[2] + g[2] % cl.m[2]) * cl.m[1] + g[1] % cl.m[1]) * cl.m[0] + g[0] % cl.m[0];
}

// Block index of neighbour d (0 = itself, 1 + 2 mu forward, 2 + 2 mu backward) of the
// aggregate with block coordinates g.
__device__ __forceinline__ int64_t mg_neighbour(const int G[4], const int g[4], int d) {
    if (d == 0) return block_index(G, g);
    const int mu = (d - 1) >> 1;
    int h[4] = {g[0], g[1], g[2], g[3]};
    h[mu] = (d & 1) ? (h[mu] + 1 == G[mu] ? 0 : h[mu] + 1) : (h[mu] == 0 ? G[mu] - 1 : h[mu] - 1);
    return block_index(G, h);
}

// Sum of N doubles over the workgroup (blockDim.x a multiple of 64); every thread gets
// the totals. lds holds (blockDim.x / 64) * N doubles.
template <int N>
__device__ __forceinline__ void wg_sum(double (&v)[N], double *lds) {
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) lds[w * N + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double t = 0;
        for (int q = 0; q < nw; ++q) t += lds[q * N + k];
        v[k] = t;
    }
    __syncthreads();
}

// Sum of the first nval of N doubles over the workgroup, written by threads t < nval to
// out[t * stride] (partials of one workgroup). lds holds (blockDim.x / 64) * N doubles.
template <int N>
__device__ __forceinline__ void wg_sum_store(double (&v)[N], double *lds, int nval, double *out, int64_t stride) {
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k < nval)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k < nval) lds[w * N + k] = v[k];
    __syncthreads();
    if ((int)threadIdx.x < nval) {
        double t = 0;
        for (int q = 0; q < nw; ++q) t += lds[q * N + threadIdx.x];
        out[(int64_t)threadIdx.x * stride] = t;
    }
}

// FP64 site component c (complex) of a block-tiled spinor field.
__device__ __forceinline__ dv2 ld64(const double *f, int64_t bp, int c, int s, int Vbh) {
    return reinterpret_cast<const dv2 *>(f)[(bp * 12 + c) * Vbh + s];
}
__device__ __forceinline__ void st64(double *f, int64_t bp, int c, int s, int Vbh, dv2 x) {
    reinterpret_cast<dv2 *>(f)[(bp * 12 + c) * Vbh + s] = x;
}
// The 6 complex components of chirality ch of site (bp, s) of the FP32 field P_j.
__device__ __forceinline__ void ldP(const float *P, int64_t bp, int ch, int s, int Vbh, float (&re)[6],
                                    float (&im)[6]) {
    const float4 *p = reinterpret_cast<const float4 *>(P);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const float4 x = p[(bp * 6 + 3 * ch + v) * Vbh + s];
        re[2 * v] = x.x;
        im[2 * v] = x.y;
        re[2 * v + 1] = x.z;
        im[2 * v + 1] = x.w;
    }
}

}  // namespace

// ---------------------------------------------------------------- set-up kernels

// In place, per aggregate and chirality: modified Gram-Schmidt with one
// reorthogonalisation pass over the nvec FP64 fields (field j at w + j * V * 24).
__global__ __launch_bounds__(512) void mg_orth_kernel(double *w, int nvec, int64_t V, int Vbh) {
    __shared__ double lds[8 * 2];
    const int tid = threadIdx.x;
    const bool act = tid < 2 * Vbh;
    const int p = act ? tid / Vbh : 0, s = act ? tid % Vbh : 0;
    const int64_t bp = 2 * (int64_t)blockIdx.x + p;
    for (int ch = 0; ch < 2; ++ch)
        for (int j = 0; j < nvec; ++j) {
            double *fj = w + (int64_t)j * V * 24;
            dv2 x[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) x[c] = act ? ld64(fj, bp, 6 * ch + c, s, Vbh) : dv2{0.0, 0.0};
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i < j; ++i) {
                    const double *fi = w + (int64_t)i * V * 24;
                    dv2 q[6];
                    double d[2] = {0.0, 0.0};
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        q[c] = act ? ld64(fi, bp, 6 * ch + c, s, Vbh) : dv2{0.0, 0.0};
                        d[0] += q[c].x * x[c].x + q[c].y * x[c].y;
                        d[1] += q[c].x * x[c].y - q[c].y * x[c].x;
                    }
                    wg_sum<2>(d, lds);
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        x[c].x -= d[0] * q[c].x - d[1] * q[c].y;
                        x[c].y -= d[0] * q[c].y + d[1] * q[c].x;
                    }
                }
            double n[1] = {0.0};
#pragma unroll
            for (int c = 0; c < 6; ++c) n[0] += x[c].x * x[c].x + x[c].y * x[c].y;
            wg_sum<1>(n, lds);
            const double inv = n[0] > 0 ? 1.0 / sqrt(n[0]) : 0.0;
            if (act)
#pragma unroll
                for (int c = 0; c < 6; ++c) st64(fj, bp, 6 * ch + c, s, Vbh, x[c] * inv);
        }
}

hipError_t launch_mg_orth(const Geom &geo, double *w, int nvec, hipStream_t st) {
    if (nvec < 1 || nvec > MG_NVEC_MAX) return hipErrorInvalidValue;
    const int nt = (2 * geo.Vbh + 63) / 64 * 64;
    hipLaunchKernelGGL(mg_orth_kernel, dim3((unsigned)geo.Nd), dim3(nt), 0, st, w, nvec, geo.V, geo.Vbh);
    return hipGetLastError();
}

// Scatter one probe: R[col][b][row] = (P^H M P e_col)(b) for the unit coarse vectors of
// columns k0 + col on the aggregates of colour q. Aggregates of one colour differ by a
// multiple of m_mu in every direction, with m_mu >= 3 or m_mu = G_mu, so among an
// aggregate and its eight neighbours at most one distinct aggregate has colour q, and
// R(b) is that aggregate's block column (D_c vanishes between aggregates that are not
// neighbours). With a block-grid extent of 2 the forward and backward neighbour coincide;
// the first match (forward) then takes both couplings.
__global__ void mg_scatter_kernel(const float2 *R, int ncol, int k0, int K, int q, MgColouring cl, Geom geo,
                                  float2 *Dc) {
    const int64_t n = geo.Nd * ncol * K;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int row = (int)(t % K);
    const int col = (int)(t / K % ncol);
    const int64_t b = t / ((int64_t)K * ncol);
    int g[4];
    block_coords(geo.G, b, g);
    for (int d = 0; d < 9; ++d) {
        int h[4] = {g[0], g[1], g[2], g[3]};
        if (d > 0) {
            const int mu = (d - 1) >> 1;
            h[mu] = (d & 1) ? (h[mu] + 1) % geo.G[mu] : (h[mu] + geo.G[mu] - 1) % geo.G[mu];
        }
        if (mg_colour(h, cl) == q) {
            Dc[((b * 9 + d) * K + k0 + col) * K + row] = R[((int64_t)col * geo.Nd + b) * K + row];
            return;
        }
    }
}

hipError_t launch_mg_scatter(const Geom &geo, const float2 *R, int ncol, int k0, int K, int q,
                             const MgColouring &cl, float2 *Dc, hipStream_t st) {
    const int64_t n = geo.Nd * ncol * K;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(mg_scatter_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, R, ncol, k0, K, q,
                       cl, geo, Dc);
    return hipGetLastError();
}

int mg_colour_of(const int g[4], const MgColouring &cl) { return mg_colour(g, cl); }

// ---------------------------------------------------------------- fine-grid kernels

// out(rhs)[b][k] = (P^H in(rhs))(b)[k] for one aggregate b per workgroup. in: FP64
// block-tiled spinors of the listed rhs at in + rhs * in_stride; out FP32 complex at
// out + rhs * out_stride. FP64 accumulation.
template <int NV>
__global__ __launch_bounds__(512) void mg_restrict_kernel(const double *in, int64_t in_stride, const float *P,
                                                           int64_t V, int Vbh, float2 *out, int64_t out_stride,
                                                           const int *active) {
    __shared__ double lds[8 * 2 * NV];
    const int tid = threadIdx.x;
    const bool act = tid < 2 * Vbh;
    const int p = act ? tid / Vbh : 0, s = act ? tid % Vbh : 0;
    const int64_t b = blockIdx.x, bp = 2 * b + p;
    const int rhs = active ? active[blockIdx.y] : (int)blockIdx.y;
    const double *r = in + (int64_t)rhs * in_stride;
    float2 *o = out + (int64_t)rhs * out_stride + b * (2 * NV);
    for (int ch = 0; ch < 2; ++ch) {
        dv2 x[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) x[c] = act ? ld64(r, bp, 6 * ch + c, s, Vbh) : dv2{0.0, 0.0};
        double acc[2 * NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            float pr[6], pi[6];
            if (act) ldP(P + (int64_t)j * V * 24, bp, ch, s, Vbh, pr, pi);
            double are = 0, aim = 0;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double qr = act ? (double)pr[c] : 0.0, qi = act ? (double)pi[c] : 0.0;
                are += qr * x[c].x + qi * x[c].y;
                aim += qr * x[c].y - qi * x[c].x;
            }
            acc[2 * j] = are;
            acc[2 * j + 1] = aim;
        }
        wg_sum<2 * NV>(acc, lds);
        if (tid == 0)
#pragma unroll
            for (int j = 0; j < NV; ++j) o[ch * NV + j] = make_float2((float)acc[2 * j], (float)acc[2 * j + 1]);
    }
}

// out(rhs) = P e(rhs) on one aggregate per workgroup, FP64 output. The coarse vector e
// on the aggregate is either
//   probe (q >= 0): 1 in column k0 + rhs on aggregates of colour q, else 0,
//   the coarse vector basis(rhs) itself (coef null), or
//   a combination sum_{i < nb} coef(rhs)[i] basis(rhs)[i] of coarse vectors.
struct MgCoarseSrc {
    const float2 *basis;   // basis(rhs)[i] at basis + rhs * bstride + i * vstride
    int64_t bstride, vstride;
    const double *coef;    // complex coef(rhs)[i] at coef + rhs * cstride + 2 i (null: basis(rhs) itself)
    int64_t cstride;
    int nb;
    int q, k0;             // probe colour (q < 0: no probe) and first column
    MgColouring cl;
};

template <int NV>
__global__ __launch_bounds__(512) void mg_prolong_kernel(MgCoarseSrc src, const float *P, Geom geo, double *out,
                                                          int64_t out_stride, const int *active) {
    constexpr int K = 2 * NV;
    __shared__ float2 e[K];
    const int tid = threadIdx.x;
    const int Vbh = geo.Vbh;
    const bool act = tid < 2 * Vbh;
    const int p = act ? tid / Vbh : 0, s = act ? tid % Vbh : 0;
    const int64_t b = blockIdx.x, bp = 2 * b + p;
    const int rhs = active ? active[blockIdx.y] : (int)blockIdx.y;
    if (tid < K) {
        float2 v = make_float2(0.f, 0.f);
        if (src.q >= 0) {
            int g[4];
            block_coords(geo.G, b, g);
            if (mg_colour(g, src.cl) == src.q && tid == src.k0 + rhs) v.x = 1.f;
        } else if (!src.coef) {  // a plain coarse vector
            v = src.basis[(int64_t)rhs * src.bstride + b * K + tid];
        } else {
            const float2 *bs = src.basis + (int64_t)rhs * src.bstride + b * K + tid;
            const double *cf = src.coef + (int64_t)rhs * src.cstride;
            double vr = 0, vi = 0;
            for (int i = 0; i < src.nb; ++i) {
                const float2 x = bs[(int64_t)i * src.vstride];
                vr += cf[2 * i] * x.x - cf[2 * i + 1] * x.y;
                vi += cf[2 * i] * x.y + cf[2 * i + 1] * x.x;
            }
            v = make_float2((float)vr, (float)vi);
        }
        e[tid] = v;
    }
    __syncthreads();
    if (!act) return;
    double *o = out + (int64_t)rhs * out_stride;
    for (int ch = 0; ch < 2; ++ch) {
        double yr[6] = {0, 0, 0, 0, 0, 0}, yi[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            float pr[6], pi[6];
            ldP(P + (int64_t)j * geo.V * 24, bp, ch, s, Vbh, pr, pi);
            const float2 c = e[ch * NV + j];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                yr[k] += (double)c.x * pr[k] - (double)c.y * pi[k];
                yi[k] += (double)c.x * pi[k] + (double)c.y * pr[k];
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) st64(o, bp, 6 * ch + k, s, Vbh, dv2{yr[k], yi[k]});
    }
}

template <int NV>
static hipError_t restrict_nv(const Geom &geo, const double *in, int64_t in_stride, const float *P, float2 *out,
                              int64_t out_stride, const int *active, int nact, hipStream_t st) {
    const int nt = (2 * geo.Vbh + 63) / 64 * 64;
    hipLaunchKernelGGL(mg_restrict_kernel<NV>, dim3((unsigned)geo.Nd, (unsigned)nact), dim3(nt), 0, st, in,
                       in_stride, P, geo.V, geo.Vbh, out, out_stride, active);
    return hipGetLastError();
}
template <int NV>
static hipError_t prolong_nv(const Geom &geo, const MgCoarseSrc &src, const float *P, double *out,
                             int64_t out_stride, const int *active, int nact, hipStream_t st) {
    const int nt = (2 * geo.Vbh + 63) / 64 * 64;
    hipLaunchKernelGGL(mg_prolong_kernel<NV>, dim3((unsigned)geo.Nd, (unsigned)nact), dim3(nt), 0, st, src, P, geo,
                       out, out_stride, active);
    return hipGetLastError();
}

#define MG_NV_SWITCH(nvec, CALL)   \
    switch (nvec) {                \
        case 2: return CALL(2);    \
        case 4: return CALL(4);    \
        case 6: return CALL(6);    \
        case 8: return CALL(8);    \
        case 10: return CALL(10);  \
        case 12: return CALL(12);  \
        case 14: return CALL(14);  \
        case 16: return CALL(16);  \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_mg_restrict(const Geom &geo, int nvec, const double *in, int64_t in_stride, const float *P,
                              float2 *out, int64_t out_stride, const int *active, int nact, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
#define MG_R(NV) restrict_nv<NV>(geo, in, in_stride, P, out, out_stride, active, nact, st)
    MG_NV_SWITCH(nvec, MG_R)
#undef MG_R
}

hipError_t launch_mg_prolong_basis(const Geom &geo, int nvec, const float *P, const float2 *basis, int64_t bstride,
                                   int64_t vstride, const double *coef, int64_t cstride, int nb, double *out,
                                   int64_t out_stride, const int *active, int nact, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    MgCoarseSrc src{};
    src.basis = basis;
    src.bstride = bstride;
    src.vstride = vstride;
    src.coef = coef;
    src.cstride = cstride;
    src.nb = nb;
    src.q = -1;
#define MG_P(NV) prolong_nv<NV>(geo, src, P, out, out_stride, active, nact, st)
    MG_NV_SWITCH(nvec, MG_P)
#undef MG_P
}

hipError_t launch_mg_prolong_probe(const Geom &geo, int nvec, const float *P, int q, const MgColouring &cl, int k0,
                                   int ncol, double *out, hipStream_t st) {
    MgCoarseSrc src{};
    src.q = q;
    src.k0 = k0;
    src.cl = cl;
#define MG_Q(NV) prolong_nv<NV>(geo, src, P, out, geo.V * 24, nullptr, ncol, st)
    MG_NV_SWITCH(nvec, MG_Q)
#undef MG_Q
}

// y(rhs) += a(rhs) x(rhs) over whole block-tiled spinor fields: x FP64, y FP64 or FP32,
// a(rhs) = alpha * scale[rhs * sstride] (alpha alone if scale is null). One thread per
// 16-byte vector of y.
template <class TY>
__global__ void mg_axpy_kernel(TY *y, int64_t ystride, const double *x, int64_t xstride, double alpha,
                               const double *scale, int sstride, const int *active, int64_t nvec16, int Vbh) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nvec16) return;
    const int rhs = active ? active[blockIdx.y] : (int)blockIdx.y;
    const double a = scale ? alpha * scale[(int64_t)rhs * sstride] : alpha;
    const dv2 *xs = reinterpret_cast<const dv2 *>(x + (int64_t)rhs * xstride);
    if constexpr (sizeof(TY) == 8) {
        dv2 *ys = reinterpret_cast<dv2 *>(y + (int64_t)rhs * ystride);
        ys[t] += a * xs[t];
    } else {
        // FP32 vector t = ((bp * 6 + v) * Vbh + s) holds the complex components 2v, 2v+1
        // that sit in FP64 vectors (bp * 12 + 2v) * Vbh + s and the next component
        const int s = (int)(t % Vbh);
        const int64_t u = t / Vbh;
        const int v = (int)(u % 6);
        const int64_t bp = u / 6;
        float4 *ys = reinterpret_cast<float4 *>(y + (int64_t)rhs * ystride);
        const dv2 x0 = xs[(bp * 12 + 2 * v) * Vbh + s], x1 = xs[(bp * 12 + 2 * v + 1) * Vbh + s];
        float4 w = ys[t];
        w.x = (float)((double)w.x + a * x0.x);
        w.y = (float)((double)w.y + a * x0.y);
        w.z = (float)((double)w.z + a * x1.x);
        w.w = (float)((double)w.w + a * x1.y);
        ys[t] = w;
    }
}

hipError_t launch_mg_axpy(const Geom &geo, Fld y, int64_t ystride, const double *x, int64_t xstride, double alpha,
                          const double *scale, int sstride, const int *active, int nact, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    if (y.prec == P64) {
        const int64_t n = geo.V * 12;
        hipLaunchKernelGGL(mg_axpy_kernel<double>, dim3((unsigned)((n + 255) / 256), (unsigned)nact), dim3(256), 0,
                           st, (double *)y.data, ystride, x, xstride, alpha, scale, sstride, active, n, geo.Vbh);
    } else if (y.prec == P32) {
        const int64_t n = geo.V * 6;
        hipLaunchKernelGGL(mg_axpy_kernel<float>, dim3((unsigned)((n + 255) / 256), (unsigned)nact), dim3(256), 0, st,
                           (float *)y.data, ystride, x, xstride, alpha, scale, sstride, active, n, geo.Vbh);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- coarse GMRES

// Workgroup tiling of the coarse kernels. The operator kernels give every aggregate's K
// rows sixteen threads each, one per column group: thread g of a row takes columns g,
// g + 16 of each of the nine blocks (the aggregate and its eight neighbours), at most 18
// terms, all of whose loads are in flight together. 512 threads cover 32 / K aggregates,
// so the stencil (18 MB on a 16^3 x 32 lattice with K = 32) streams from many CUs. The
// Gram-Schmidt kernels of the two-launch form take 256 / K aggregates per 256-thread
// workgroup: every one of their workgroups re-sums all partials of the previous kernel,
// so their count is kept small (their re-reads grow as the product of both counts).
constexpr int MG_AWG = 512, MG_ALANES = 32, MG_AGRP = MG_AWG / MG_ALANES, MG_GWG = 256;
constexpr int MG_CPG = (2 * MG_NVEC_MAX + MG_AGRP - 1) / MG_AGRP;  // columns per group and block
static_assert(MG_IMAX <= 2 * MG_AGRP, "the operator kernel's column groups take two basis vectors each");
void mg_coarse_tiling(const Geom &geo, int K, int *nwa, int *nwc) {
    const int ta = MG_ALANES / K > 0 ? MG_ALANES / K : 1, tc = MG_GWG / K > 0 ? MG_GWG / K : 1;
    *nwa = (int)((geo.Nd + ta - 1) / ta);
    *nwc = (int)((geo.Nd + tc - 1) / tc);
}

namespace {

// Sum of value v over n partials (stride 1) by one wave in a fixed order: lane l adds
// partials l, l + 64, ..., then a butterfly over the lanes; every lane gets the total.
__device__ __forceinline__ double wave_sum_parts(const double *part, int n) {
    const int lane = threadIdx.x & 63;
    // partials lane, lane + 64, lane + 128, lane + 192 by unconditional loads (clamped to
    // partial 0, written and finite, and multiplied by zero past n), so that none waits
    // behind a branch; then the rest
    double x[4], t = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = part[lane + 64 * q < n ? lane + 64 * q : 0];
#pragma unroll
    for (int q = 0; q < 4; ++q) t += x[q] * (lane + 64 * q < n ? 1.0 : 0.0);
    for (int q = lane + 4 * 64; q < n; q += 64) t += part[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    return t;
}

// The totals of nval <= 2 MG_IMAX values (value v's n partials at part + v * pstride)
// into h[v] in LDS in a fixed order: value v by wave v mod NW (blockDim.x = 64 NW), whose
// lane l adds partials l, l + 64, ... (the loads of 256 partials in flight together),
// then one butterfly per value; then a barrier.
template <int NW, int NV = 2 * MG_IMAX>
__device__ __forceinline__ void load_totals(const double *part, int64_t pstride, int n, int nval, double *h) {
    constexpr int PER = (NV + NW - 1) / NW;  // nval <= NV
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double acc[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) acc[u] = 0.0;
    for (int q0 = 0; q0 < n; q0 += 4 * 64) {
        // every load unconditional, so that all are in flight together: an index out of
        // range reads partial 0 of value 0 (written and finite) and adds it times zero,
        // which leaves the sum's bits unchanged
        double x[4][PER];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int q = q0 + 64 * qq + lane;
                const bool in = q < n && w + NW * u < nval;
                x[qq][u] = part[(int64_t)(in ? w + NW * u : 0) * pstride + (in ? q : 0)];
            }
        __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the sums
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int q = q0 + 64 * qq + lane;
                acc[u] += x[qq][u] * (q < n && w + NW * u < nval ? 1.0 : 0.0);
            }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u)
        if (w + NW * u < nval) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off, 64);
            if (lane == 0) h[w + NW * u] = acc[u];
        }
    __syncthreads();
}

__device__ __forceinline__ double *pd_of(const MgGmres &G, int rhs, int pass) {
    return G.pd + ((int64_t)rhs * 2 + pass) * 2 * MG_IMAX * G.pstride;
}
__device__ __forceinline__ double *pn_of(const MgGmres &G, int rhs, int i) {
    return G.pn + ((int64_t)rhs * (MG_IMAX + 1) + i) * G.pstride;
}

// Thread layout of the operator kernels: column group g (0..MG_AGRP-1) of row a of
// aggregate b; act: the row exists.
struct CoarseRow {
    int g, r, a;
    int64_t b;
    bool act;
    __device__ __forceinline__ CoarseRow(const MgGmres &G) {
        const int K = G.K, ta = MG_ALANES / K > 0 ? MG_ALANES / K : 1;
        g = threadIdx.x / MG_ALANES;
        r = threadIdx.x % MG_ALANES;
        const int bl = r / K;
        a = r - bl * K;
        b = (int64_t)blockIdx.x * ta + bl;
        act = bl < ta && b < G.Nd;
    }
};

// This thread's part of row a of (D_c x) for aggregate b: columns g, g + MG_AGRP, ... of
// the nine blocks in block order, added to (yr, yi). Every load is issued before the
// sums.
__device__ __forceinline__ void coarse_row_part(const MgGmres &G, const CoarseRow &w, const float2 *x, double &yr,
                                                double &yi) {
    const int K = G.K;
    int gc[4];
    block_coords(G.grid, w.b, gc);
    // all loads first (unconditional, so that none waits for another: a column past K
    // reads column 0 and is multiplied by zero), then the sums in block and column order
    float2 m[9][MG_CPG], xv[9][MG_CPG];
#pragma unroll
    for (int d = 0; d < 9; ++d) {
        const int64_t nb = mg_neighbour(G.grid, gc, d);
        const float2 *dcol = G.Dc + ((w.b * 9 + d) * K) * K + w.a;
        const float2 *xn = x + nb * K;
#pragma unroll
        for (int t = 0; t < MG_CPG; ++t) {
            const int c = w.g + MG_AGRP * t;
            m[d][t] = dcol[(int64_t)(c < K ? c : 0) * K];
            xv[d][t] = xn[c < K ? c : 0];
        }
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the sums
#pragma unroll
    for (int d = 0; d < 9; ++d)
#pragma unroll
        for (int t = 0; t < MG_CPG; ++t) {
            const float f = w.g + MG_AGRP * t < K ? 1.f : 0.f;
            const float mr = m[d][t].x * f, mi = m[d][t].y * f;
            yr += (double)mr * xv[d][t].x - (double)mi * xv[d][t].y;
            yi += (double)mr * xv[d][t].y + (double)mi * xv[d][t].x;
        }
}

// Row r of D_c x from the column groups' parts in ys (after a barrier), summed in group
// order.
__device__ __forceinline__ void coarse_row_total(const double (&ys)[2][MG_AGRP][MG_ALANES], int r, double &yr,
                                                 double &yi) {
    yr = yi = 0;
#pragma unroll
    for (int q = 0; q < MG_AGRP; ++q) {
        yr += ys[0][q][r];
        yi += ys[1][q][r];
    }
}

}  // namespace

// |v_0|^2 partials of every listed system (v_0 = the restricted right-hand side).
__global__ __launch_bounds__(MG_GWG) void mg_cinit_kernel(MgGmres G) {
    const int rhs = G.active[blockIdx.y];
    const int K = G.K, tc = MG_GWG / K > 0 ? MG_GWG / K : 1;
    const int bl = threadIdx.x / K, a = threadIdx.x - bl * K;
    const int64_t b = (int64_t)blockIdx.x * tc + bl;
    __shared__ double lds[MG_GWG / 64];
    double n[1] = {0.0};
    if (bl < tc && b < G.Nd) {
        const float2 x = G.basis[(int64_t)rhs * G.bstride + b * K + a];
        n[0] = (double)x.x * x.x + (double)x.y * x.y;
    }
    wg_sum_store<1>(n, lds, 1, pn_of(G, rhs, 0) + blockIdx.x, 1);
}

// Arnoldi step j, pass 0: w = D_c (s_j v_j) into basis slot j + 1 and the partials of
// <v_i, w>, i <= j (the Gram-Schmidt kernel applies s_i to their totals). s_j = 1 / |v_j|
// from the norm partials of v_j. Every thread issues its stencil loads and the rows of
// its two basis vectors (i = g and g + MG_AGRP) at once; after one barrier each thread
// sums its row of w from the column groups' parts, and each group's two dot products
// are summed over the 32 rows by a half-wave butterfly.
__global__ __launch_bounds__(MG_AWG) __attribute__((amdgpu_waves_per_eu(1, 4))) void mg_capply_kernel(MgGmres G,
                                                                                                      int j) {
    __shared__ double ys[2][MG_AGRP][MG_ALANES];
    const int rhs = G.active[blockIdx.y];
    const int K = G.K;
    const CoarseRow w(G);
    const float2 *vb = G.basis + (int64_t)rhs * G.bstride;
    const float2 *vj = vb + (int64_t)j * G.vstride;
    float2 *wout = const_cast<float2 *>(vb) + (int64_t)(j + 1) * G.vstride;
    // unconditional loads with clamped indices: for i > j or a missing row they read a
    // stored row whose products are not kept
    const int64_t row = w.act ? w.b * K + w.a : 0;
    float2 v[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = w.g + MG_AGRP * u;
        v[u] = vb[(int64_t)(i <= j ? i : j) * G.vstride + row];
    }
    // |v_j|^2 by every wave (fixed order, as wave_sum_parts): partial `lane` loaded with
    // the stencil (clamped, times zero past nwc), the rest and the butterfly after it
    const double *pnj = pn_of(G, rhs, j);
    const int lane = threadIdx.x & 63;
    double nj = pnj[lane < G.nwc ? lane : 0] * (lane < G.nwc ? 1.0 : 0.0);
    double yr = 0, yi = 0;  // this thread's part of (D_c v_j) row a of aggregate b
    if (w.act) coarse_row_part(G, w, vj, yr, yi);
    ys[0][w.g][w.r] = yr;
    ys[1][w.g][w.r] = yi;
    for (int q = lane + 64; q < G.nwc; q += 64) nj += pnj[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nj += __shfl_xor(nj, off, 64);
    __syncthreads();
    const double sj = nj > 0 ? 1.0 / sqrt(nj) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        G.sc[(int64_t)rhs * (MG_IMAX + 1) + j] = sj;
        const double h = sqrt(nj > 0 ? nj : 0.0);
        if (j == 0) {
            G.beta[rhs] = h;
        } else {  // h_{j,j-1}
            double *Hc = G.H + (int64_t)rhs * (MG_IMAX + 1) * MG_IMAX * 2 + 2 * (int64_t)(j - 1) * (MG_IMAX + 1);
            Hc[2 * j] = h;
            Hc[2 * j + 1] = 0.0;
        }
    }
    coarse_row_total(ys, w.r, yr, yi);
    yr *= sj;
    yi *= sj;
    if (w.act) {
        const float2 wf = make_float2((float)yr, (float)yi);
        if (w.g == 0) wout[w.b * K + w.a] = wf;
        yr = wf.x;  // the dot products see the stored vector
        yi = wf.y;
    } else {
        yr = yi = 0;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = w.g + MG_AGRP * u;
        double pr = (double)v[u].x * yr + (double)v[u].y * yi;
        double pi = (double)v[u].x * yi - (double)v[u].y * yr;
#pragma unroll
        for (int off = MG_ALANES / 2; off > 0; off >>= 1) {  // the 32 rows of this group
            pr += __shfl_xor(pr, off, 64);
            pi += __shfl_xor(pi, off, 64);
        }
        if (w.r == 0 && i <= j) {
            double *pd = pd_of(G, rhs, 0) + blockIdx.x;
            pd[(int64_t)(2 * i) * G.pstride] = pr;
            pd[(int64_t)(2 * i + 1) * G.pstride] = pi;
        }
    }
}

// Arnoldi step j, a correction pass: w -= sum_i h_i s_i v_i with h_i = s_i t_i and t the
// totals of the partials of pass `src` (0: the operator kernel's <v_i, w>, 1: a second
// pass's); then either the partials of <v_i, w> for a further pass (norm = 0) or of
// |w|^2 (norm = 1). Workgroup 0 sets (src 0) or adds (src 1) h into column j of the
// Hessenberg matrix.
__global__ __launch_bounds__(MG_GWG) void mg_cgs_kernel(MgGmres G, int j, int src, int norm) {
    __shared__ double h[2 * MG_IMAX];
    __shared__ double lds[(MG_GWG / 64) * 2 * MG_IMAX];
    const int rhs = G.active[blockIdx.y];
    const int K = G.K, tc = MG_GWG / K > 0 ? MG_GWG / K : 1;
    const int bl = threadIdx.x / K, a = threadIdx.x - bl * K;
    const int64_t b = (int64_t)blockIdx.x * tc + bl;
    const bool act = bl < tc && b < G.Nd;
    const float2 *vb = G.basis + (int64_t)rhs * G.bstride;
    float2 *w = const_cast<float2 *>(vb) + (int64_t)(j + 1) * G.vstride;
    // this thread's rows of w and of the basis, loaded before the partial sums
    // (unconditional loads with clamped indices: for i > j or a missing row they read a
    // stored row that enters with a zero coefficient or is not kept)
    const int64_t row = act ? b * K + a : 0;
    const float2 w0 = w[row];
    float2 vi[MG_IMAX];
#pragma unroll
    for (int i = 0; i < MG_IMAX; ++i) vi[i] = vb[(int64_t)(i <= j ? i : j) * G.vstride + row];
    // s_i in lane i of every wave (s_0 .. s_j are written; lanes past j read s_j)
    const double *sc = G.sc + (int64_t)rhs * (MG_IMAX + 1);
    const int lane = threadIdx.x & 63;
    const double s_lane = sc[lane <= j ? lane : j];
    load_totals<MG_GWG / 64>(pd_of(G, rhs, src), G.pstride, src == 0 ? G.nwa : G.nwc, 2 * (j + 1), h);
    if (blockIdx.x == 0 && (int)threadIdx.x < 2 * (j + 1)) {
        double *Hc = G.H + (int64_t)rhs * (MG_IMAX + 1) * MG_IMAX * 2 + 2 * (int64_t)j * (MG_IMAX + 1);
        Hc[threadIdx.x] = (src == 0 ? 0.0 : Hc[threadIdx.x]) + h[threadIdx.x] * __shfl(s_lane, threadIdx.x >> 1, 64);
    }
    double yr = w0.x, yi = w0.y;
#pragma unroll
    for (int i = 0; i < MG_IMAX; ++i) {  // the terms i > j are zeros
        const double si = __shfl(s_lane, i, 64);
        const double cr = i <= j ? h[2 * i] * si * si : 0.0, ci = i <= j ? h[2 * i + 1] * si * si : 0.0;
        yr -= cr * vi[i].x - ci * vi[i].y;
        yi -= cr * vi[i].y + ci * vi[i].x;
    }
    if (act) w[b * K + a] = make_float2((float)yr, (float)yi);
    yr = act ? (double)(float)yr : 0.0;
    yi = act ? (double)(float)yi : 0.0;
    if (!norm) {
        double acc[2 * MG_IMAX];
#pragma unroll
        for (int i = 0; i < MG_IMAX; ++i) {
            acc[2 * i] = acc[2 * i + 1] = 0.0;
            if (i <= j && act) {
                acc[2 * i] = (double)vi[i].x * yr + (double)vi[i].y * yi;
                acc[2 * i + 1] = (double)vi[i].x * yi - (double)vi[i].y * yr;
            }
        }
        wg_sum_store<2 * MG_IMAX>(acc, lds, 2 * (j + 1), pd_of(G, rhs, 1) + blockIdx.x, G.pstride);
    } else {
        double n[1] = {yr * yr + yi * yi};
        wg_sum_store<1>(n, lds, 1, pn_of(G, rhs, j + 1) + blockIdx.x, 1);
    }
}

// Arnoldi step j of a cycle in one launch (classical Gram-Schmidt, one pass). The basis
// holds v_i (unnormalised, q_i = s_i v_i with s_i = 1 / |v_i|); u_j = D_c v_{j-1} is kept
// unscaled in one of two slots after the basis. Step j
//  1. sums the partials of step j - 1 (every workgroup for itself, in a fixed order):
//     |v_{j-1}|^2, so s_{j-1}, and t_i = <v_i, u_j>, so h_{i,j-1} = s_i s_{j-1} t_i;
//  2. forms v_j = s_{j-1} u_j - sum_{i<j} h_{i,j-1} s_i v_i (v_0: the cycle's start) at
//     the rows of every aggregate of the workgroup and of their eight neighbours, into
//     LDS, and stores its own rows into basis slot j;
//  3. writes the partials of |v_j|^2 and, unless TAIL, applies the stencil to v_j from
//     LDS: u_{j+1} = D_c v_j, stored, and the partials of <v_i, u_{j+1}>, i <= j.
// Workgroup 0 writes s_{j-1}, column j - 1 of the Hessenberg matrix and its entry
// h_{j-1,j-2} = |v_{j-1}| (beta for j = 1). The TAIL launch (j = k) ends the cycle: it
// leaves |v_k|^2 in partials for the least-squares kernel. Every load of a thread is
// issued before its sums (clamped indices; values outside the ranges are multiplied by
// zero or not kept); JB >= j bounds the basis vectors a step loads.
template <bool TAIL, int JB>
__global__ __launch_bounds__(MG_AWG) __attribute__((amdgpu_waves_per_eu(1, 2))) void mg_carnoldi_kernel(MgGmres G,
                                                                                                       int j) {
    constexpr int NW = MG_AWG / 64, NE = 9 * MG_ALANES;  // LDS entries: 9 blocks x 32 rows
    __shared__ float2 xs[NE];
    __shared__ double ys[2][MG_AGRP][MG_ALANES];
    __shared__ double h[2 * MG_IMAX];
    const int rhs = G.active[blockIdx.y];
    const int K = G.K, ta = MG_ALANES / K > 0 ? MG_ALANES / K : 1;
    const int lane = threadIdx.x & 63;
    const CoarseRow w(G);
    float2 *vb = G.basis + (int64_t)rhs * G.bstride;
    const float2 *uj = vb + (int64_t)(MG_IMAX + 1 + (j & 1)) * G.vstride;
    float2 *un = vb + (int64_t)(MG_IMAX + 1 + ((j + 1) & 1)) * G.vstride;
    const double *sc = G.sc + (int64_t)rhs * (MG_IMAX + 1);
    const int jp = j > 0 ? j - 1 : 0;  // the previous step (clamped)

    // ---- loads
    // entry e of the LDS block: (aggregate bl, neighbour block d, row c)
    const int e = threadIdx.x;
    const int ebl = e / (9 * K), erem = e - ebl * 9 * K, ed = erem / K, ec = erem - ed * K;
    const int64_t eb = (int64_t)blockIdx.x * ta + ebl;
    const bool eact = e < NE && ebl < ta && eb < G.Nd;
    int64_t erow = 0;
    {  // neighbour ed of aggregate eb without indexing the grid by a per-thread direction
        const int gg[4] = {G.grid[0], G.grid[1], G.grid[2], G.grid[3]};
        int gc[4], hc[4];
        block_coords(gg, eact ? eb : 0, gc);
        const int mu = (ed - 1) >> 1;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int up = gc[m] + 1 == gg[m] ? 0 : gc[m] + 1, dn = gc[m] == 0 ? gg[m] - 1 : gc[m] - 1;
            hc[m] = ed > 0 && m == mu ? ((ed & 1) ? up : dn) : gc[m];
        }
        erow = eact ? block_index(gg, hc) * K + ec : 0;
    }
    const float2 ue = j > 0 ? uj[erow] : vb[erow];  // j = 0: v_0 itself
    float2 ve[JB];                                    // v_i at the entry, i < j
#pragma unroll
    for (int i = 0; i < JB; ++i) ve[i] = vb[(int64_t)(i < j ? i : jp) * G.vstride + erow];
    const double s_lane = sc[lane < jp ? lane : 0];  // s_i in lane i (i < j - 1 are written)
    const int64_t row = w.act ? w.b * K + w.a : 0;
    float2 vo[2];  // own rows of v_i, i = g and g + MG_AGRP (i < j; v_j comes from LDS)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = w.g + MG_AGRP * u;
        vo[u] = vb[(int64_t)(i < j ? i : jp) * G.vstride + row];
    }
    float2 m[9][MG_CPG];  // this thread's stencil columns (row a of aggregate b)
    if constexpr (!TAIL) {
        const int64_t bb = w.act ? w.b : 0;
#pragma unroll
        for (int d = 0; d < 9; ++d)
#pragma unroll
            for (int t = 0; t < MG_CPG; ++t) {
                const int c = w.g + MG_AGRP * t;
                m[d][t] = G.Dc[((bb * 9 + d) * K + (c < K ? c : 0)) * K + w.a];
            }
    }
    // |v_{j-1}|^2 partials lane, lane + 64, ... (the first four per lane loaded here,
    // clamped, and added times zero past nwa: the order of wave_sum_parts)
    const double *pnp = pn_of(G, rhs, jp);
    double pnr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pnr[q] = pnp[lane + 64 * q < G.nwa ? lane + 64 * q : 0];
    double np = 0;
    if (j > 0) {
        load_totals<NW, 2 * JB>(pd_of(G, rhs, jp & 1), G.pstride, G.nwa, 2 * j, h);  // ends with a barrier
#pragma unroll
        for (int q = 0; q < 4; ++q) np += pnr[q] * (lane + 64 * q < G.nwa ? 1.0 : 0.0);
        for (int q = lane + 4 * 64; q < G.nwa; q += 64) np += pnp[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) np += __shfl_xor(np, off, 64);
    }
    // ---- step j - 1's coefficients (the shuffles with every lane of the wave taking part)
    const double sp = j > 0 && np > 0 ? 1.0 / sqrt(np) : 0.0;  // s_{j-1}
    const double s_half = __shfl(s_lane, (lane >> 1) & 31, 64);  // s_{lane / 2}
    double cf[JB];  // h_{i,j-1} s_i / |...| factors: s_i^2 s_{j-1} for i < j, else 0
#pragma unroll
    for (int i = 0; i < JB; ++i) {
        const double si = i == j - 1 ? sp : __shfl(s_lane, i, 64);
        cf[i] = i < j ? si * si * sp : 0.0;
    }
    if (blockIdx.x == 0 && j > 0) {
        if (threadIdx.x == 0) {
            G.sc[(int64_t)rhs * (MG_IMAX + 1) + j - 1] = sp;
            const double hn = sqrt(np > 0 ? np : 0.0);
            if (j == 1) {
                G.beta[rhs] = hn;
            } else {  // h_{j-1,j-2}
                double *Hc = G.H + (int64_t)rhs * (MG_IMAX + 1) * MG_IMAX * 2 + 2 * (int64_t)(j - 2) * (MG_IMAX + 1);
                Hc[2 * (j - 1)] = hn;
                Hc[2 * (j - 1) + 1] = 0.0;
            }
        }
        if ((int)threadIdx.x < 2 * j) {  // h_{i,j-1} = s_i s_{j-1} t_i
            const int i = threadIdx.x >> 1;
            const double si = i == j - 1 ? sp : s_half;
            double *Hc = G.H + (int64_t)rhs * (MG_IMAX + 1) * MG_IMAX * 2 + 2 * (int64_t)(j - 1) * (MG_IMAX + 1);
            Hc[threadIdx.x] = h[threadIdx.x] * si * sp;
        }
    }
    // ---- v_j at the entry: s_{j-1} u_j - sum_i h_{i,j-1} s_i v_i (terms i >= j are zeros)
    float2 x = ue;
    if (j > 0) {
        double yr = sp * ue.x, yi = sp * ue.y;
#pragma unroll
        for (int i = 0; i < JB; ++i) {
            const double cr = i < j ? h[2 * i] * cf[i] : 0.0, ci = i < j ? h[2 * i + 1] * cf[i] : 0.0;
            yr -= cr * ve[i].x - ci * ve[i].y;
            yi -= cr * ve[i].y + ci * ve[i].x;
        }
        x = make_float2((float)yr, (float)yi);
    }
    if (e < NE) xs[e] = x;
    __syncthreads();
    // ---- own rows: store v_j (j > 0) and the partials of |v_j|^2 (group 0's 32 rows)
    const int bl = w.r / K;
    const float2 vj = w.act ? xs[bl * 9 * K + w.a] : make_float2(0.f, 0.f);
    if (j > 0 && w.act && w.g == 0) vb[(int64_t)j * G.vstride + w.b * K + w.a] = vj;
    if (w.g == 0) {
        double n = (double)vj.x * vj.x + (double)vj.y * vj.y;
#pragma unroll
        for (int off = MG_ALANES / 2; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
        if (w.r == 0) pn_of(G, rhs, j)[blockIdx.x] = n;
    }
    if constexpr (TAIL) return;
    // ---- u_{j+1} = D_c v_j from LDS: columns g, g + MG_AGRP of the nine blocks
    double yr = 0, yi = 0;
    if (w.act) {
#pragma unroll
        for (int d = 0; d < 9; ++d)
#pragma unroll
            for (int t = 0; t < MG_CPG; ++t) {
                const int c = w.g + MG_AGRP * t;
                const float f = c < K ? 1.f : 0.f;
                const float2 xv = xs[(bl * 9 + d) * K + (c < K ? c : 0)];
                const float mr = m[d][t].x * f, mi = m[d][t].y * f;
                yr += (double)mr * xv.x - (double)mi * xv.y;
                yi += (double)mr * xv.y + (double)mi * xv.x;
            }
    }
    ys[0][w.g][w.r] = yr;
    ys[1][w.g][w.r] = yi;
    __syncthreads();
    coarse_row_total(ys, w.r, yr, yi);
    if (w.act) {
        const float2 uf = make_float2((float)yr, (float)yi);
        if (w.g == 0) un[w.b * K + w.a] = uf;
        yr = uf.x;  // the dot products see the stored vector
        yi = uf.y;
    } else {
        yr = yi = 0;
    }
    // ---- partials of <v_i, u_{j+1}>, i <= j: two basis vectors per column group
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = w.g + MG_AGRP * u;
        const float2 v = i == j ? vj : vo[u];
        double pr = (double)v.x * yr + (double)v.y * yi;
        double pi = (double)v.x * yi - (double)v.y * yr;
#pragma unroll
        for (int off = MG_ALANES / 2; off > 0; off >>= 1) {  // the 32 rows of this group
            pr += __shfl_xor(pr, off, 64);
            pi += __shfl_xor(pi, off, 64);
        }
        if (w.r == 0 && i <= j) {
            double *pd = pd_of(G, rhs, j & 1) + blockIdx.x;
            pd[(int64_t)(2 * i) * G.pstride] = pr;
            pd[(int64_t)(2 * i + 1) * G.pstride] = pi;
        }
    }
}

// After k steps, one wave per system: h_{k,k-1} from the last norm partials, then
// min |beta e_1 - Hbar y| by Givens rotations with lane c holding column c of Hbar (each
// rotation is broadcast from the lane of its column and applied by all lanes), back
// substitution with a lane sum per row, and coef[i] = y_i s_i, so that the coarse
// solution is sum_i coef[i] v_i over the stored (unnormalised) basis. A zero diagonal
// after the rotations (exact breakdown) gives y_i = 0.
__global__ __launch_bounds__(64) void mg_cfinal_kernel(MgGmres G, int k) {
    const int rhs = G.active[blockIdx.x];
    const int lane = threadIdx.x;
    const double nk = wave_sum_parts(pn_of(G, rhs, k), G.fused ? G.nwa : G.nwc);
    const double *Hm = G.H + (int64_t)rhs * (MG_IMAX + 1) * MG_IMAX * 2;
    const double *sc = G.sc + (int64_t)rhs * (MG_IMAX + 1);
    double hr[MG_IMAX + 1], hi[MG_IMAX + 1];  // column `lane` of Hbar, rows 0..MG_IMAX
    // Every load is unconditional and reads an entry this cycle has written (column
    // col = lane or 0, rows 0..col, and row lane + 1 where it exists); entries outside
    // the column are then multiplied by zero, so no load waits behind a branch.
    const int col = lane < k ? lane : 0;
    const bool sub = lane + 1 < k;  // h_{lane+1,lane} is stored (else it is |w_k|)
    const double *Hcol = Hm + 2 * (int64_t)col * (MG_IMAX + 1);
    const double hs = Hcol[2 * (sub ? lane + 1 : col)];
    const double hk = sqrt(nk > 0 ? nk : 0.0);
#pragma unroll
    for (int r = 0; r <= MG_IMAX; ++r) {
        const int rr = r <= col ? r : col;
        const double m = lane < k && r <= lane ? 1.0 : 0.0;
        hr[r] = Hcol[2 * rr] * m;
        hi[r] = Hcol[2 * rr + 1] * m;
        if (lane < k && r == lane + 1) hr[r] = hs * (sub ? 1.0 : 0.0) + hk * (sub ? 0.0 : 1.0);
    }
    double gr[MG_IMAX + 1], gi[MG_IMAX + 1];
#pragma unroll
    for (int r = 0; r <= MG_IMAX; ++r) gr[r] = gi[r] = 0.0;
    gr[0] = G.beta[rhs];
#pragma unroll
    for (int i = 0; i < MG_IMAX; ++i) {
        if (i < k) {
            // rotation [[c, s], [-conj(s), c]] with c a + s b = r, -conj(s) a + c b = 0 for
            // (a, b) = rows i, i + 1 of column i
            const double ar = __shfl(hr[i], i, 64), ai = __shfl(hi[i], i, 64);
            const double br = __shfl(hr[i + 1], i, 64), bi = __shfl(hi[i + 1], i, 64);
            const double na = sqrt(ar * ar + ai * ai), nb = sqrt(br * br + bi * bi);
            double c, sr, si;
            if (nb == 0.0) {
                c = 1.0;
                sr = si = 0.0;
            } else if (na == 0.0) {
                const double inb = 1.0 / nb;
                c = 0.0;
                sr = br * inb;
                si = -bi * inb;
            } else {
                const double irr = 1.0 / sqrt(na * na + nb * nb), ina = 1.0 / na;
                c = na * irr;
                const double ur = ar * ina, ui = ai * ina;  // s = (a / |a|) conj(b) / r
                sr = (ur * br + ui * bi) * irr;
                si = (ui * br - ur * bi) * irr;
            }
            const double xr = hr[i], xi = hi[i], yr = hr[i + 1], yi = hi[i + 1];
            hr[i] = c * xr + (sr * yr - si * yi);
            hi[i] = c * xi + (sr * yi + si * yr);
            hr[i + 1] = -(sr * xr + si * xi) + c * yr;
            hi[i + 1] = -(sr * xi - si * xr) + c * yi;
            const double g0r = gr[i], g0i = gi[i], g1r = gr[i + 1], g1i = gi[i + 1];
            gr[i] = c * g0r + (sr * g1r - si * g1i);
            gi[i] = c * g0i + (sr * g1i + si * g1r);
            gr[i + 1] = -(sr * g0r + si * g0i) + c * g1r;
            gi[i + 1] = -(sr * g0i - si * g0r) + c * g1i;
        }
    }
    // back substitution: lane q holds R[i][q] in (hr[i], hi[i]) and, once known, y_q
    double ylr = 0.0, yli = 0.0;
#pragma unroll
    for (int i = MG_IMAX - 1; i >= 0; --i) {
        if (i < k) {
            double pr = 0.0, pi = 0.0;
            if (lane > i && lane < k) {
                pr = hr[i] * ylr - hi[i] * yli;
                pi = hr[i] * yli + hi[i] * ylr;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                pr += __shfl_xor(pr, off, 64);
                pi += __shfl_xor(pi, off, 64);
            }
            const double dr = __shfl(hr[i], i, 64), di = __shfl(hi[i], i, 64), dd = dr * dr + di * di;
            const double tr = gr[i] - pr, ti = gi[i] - pi;
            const double idd = dd > 0 ? 1.0 / dd : 0.0;
            if (lane == i) {
                ylr = (tr * dr + ti * di) * idd;
                yli = (ti * dr - tr * di) * idd;
            }
        }
    }
    if (lane < k) {
        double *cf = G.coef + (int64_t)rhs * 2 * MG_IMAX;
        cf[2 * lane] = ylr * sc[lane];
        cf[2 * lane + 1] = yli * sc[lane];
    }
}

// Start of a restart cycle: v_0 = rc - D_c xc (v_0 = rc on the first cycle, xc = 0).
// Same tiling as the operator kernel.
__global__ __launch_bounds__(MG_AWG) __attribute__((amdgpu_waves_per_eu(1, 4))) void mg_cres_kernel(MgGmres G,
                                                                                                    int first) {
    __shared__ double ys[2][MG_AGRP][MG_ALANES];
    const int rhs = G.active[blockIdx.y];
    const int K = G.K;
    const CoarseRow w(G);
    const float2 *xc = G.xc + (int64_t)rhs * G.vstride;
    const float2 rc = w.act ? G.rc[(int64_t)rhs * G.vstride + w.b * K + w.a] : make_float2(0.f, 0.f);
    float2 *v0 = G.basis + (int64_t)rhs * G.bstride;
    if (first) {
        if (w.act && w.g == 0) v0[w.b * K + w.a] = rc;
        return;
    }
    double yr = 0, yi = 0;
    if (w.act) coarse_row_part(G, w, xc, yr, yi);
    ys[0][w.g][w.r] = yr;
    ys[1][w.g][w.r] = yi;
    __syncthreads();
    if (w.g != 0 || !w.act) return;
    coarse_row_total(ys, w.r, yr, yi);
    v0[w.b * K + w.a] = make_float2((float)(rc.x - yr), (float)(rc.y - yi));
}

// End of a restart cycle: xc = (first ? 0 : xc) + sum_{i < k} coef[i] v_i.
__global__ void mg_caccum_kernel(MgGmres G, int k, int first) {
    const int64_t n = G.Nd * G.K;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int rhs = G.active[blockIdx.y];
    const float2 *bs = G.basis + (int64_t)rhs * G.bstride + t;
    const double *cf = G.coef + (int64_t)rhs * 2 * MG_IMAX;
    float2 *xc = G.xc + (int64_t)rhs * G.vstride + t;
    double vr = first ? 0.0 : (double)xc->x, vi = first ? 0.0 : (double)xc->y;
    for (int i = 0; i < k; ++i) {
        const float2 x = bs[(int64_t)i * G.vstride];
        vr += cf[2 * i] * x.x - cf[2 * i + 1] * x.y;
        vi += cf[2 * i] * x.y + cf[2 * i + 1] * x.x;
    }
    *xc = make_float2((float)vr, (float)vi);
}

// Step j of the Arnoldi kernel (the cycle's tail for j = k) with the smallest bound on
// the basis vectors it loads.
static void launch_arnoldi(bool tail, int j, dim3 ga, hipStream_t st, const MgGmres &G) {
    static_assert(MG_IMAX == 24, "the bounds below cover MG_IMAX steps");
    if (tail) {
        if (j <= 8) hipLaunchKernelGGL((mg_carnoldi_kernel<true, 8>), ga, dim3(MG_AWG), 0, st, G, j);
        else if (j <= 16) hipLaunchKernelGGL((mg_carnoldi_kernel<true, 16>), ga, dim3(MG_AWG), 0, st, G, j);
        else hipLaunchKernelGGL((mg_carnoldi_kernel<true, 24>), ga, dim3(MG_AWG), 0, st, G, j);
    } else {
        if (j <= 8) hipLaunchKernelGGL((mg_carnoldi_kernel<false, 8>), ga, dim3(MG_AWG), 0, st, G, j);
        else if (j <= 16) hipLaunchKernelGGL((mg_carnoldi_kernel<false, 16>), ga, dim3(MG_AWG), 0, st, G, j);
        else hipLaunchKernelGGL((mg_carnoldi_kernel<false, 24>), ga, dim3(MG_AWG), 0, st, G, j);
    }
}

hipError_t launch_mg_coarse_gmres(const MgGmres &G, int nact, int k, int cycles, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    if (k < 1 || k > MG_IMAX || cycles < 1 || G.K < 2 || G.K > 2 * MG_NVEC_MAX) return hipErrorInvalidValue;
    const dim3 ga((unsigned)G.nwa, (unsigned)nact), gc((unsigned)G.nwc, (unsigned)nact);
    const int64_t n = G.Nd * G.K;
    const dim3 ge((unsigned)((n + 255) / 256), (unsigned)nact);
    for (int cyc = 0; cyc < cycles; ++cyc) {
        hipLaunchKernelGGL(mg_cres_kernel, ga, dim3(MG_AWG), 0, st, G, (int)(cyc == 0));
        if (G.fused) {  // one launch per step
            for (int j = 0; j <= k; ++j) launch_arnoldi(j == k, j, ga, st, G);
        } else {  // two launches per step
            hipLaunchKernelGGL(mg_cinit_kernel, gc, dim3(MG_GWG), 0, st, G);
            for (int j = 0; j < k; ++j) {
                hipLaunchKernelGGL(mg_capply_kernel, ga, dim3(MG_AWG), 0, st, G, j);
                hipLaunchKernelGGL(mg_cgs_kernel, gc, dim3(MG_GWG), 0, st, G, j, 0, 1);
            }
        }
        hipLaunchKernelGGL(mg_cfinal_kernel, dim3((unsigned)nact), dim3(64), 0, st, G, k);
        hipLaunchKernelGGL(mg_caccum_kernel, ge, dim3(256), 0, st, G, k, (int)(cyc == 0));
    }
    return hipGetLastError();
}

// out(rhs) = the coarse solution xc(rhs) as complex FP64 (out + rhs * ostride doubles).
__global__ void mg_solution_kernel(MgGmres G, double *out, int64_t ostride) {
    const int64_t n = G.Nd * G.K;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int rhs = G.active[blockIdx.y];
    const float2 x = G.xc[(int64_t)rhs * G.vstride + t];
    out[(int64_t)rhs * ostride + 2 * t] = x.x;
    out[(int64_t)rhs * ostride + 2 * t + 1] = x.y;
}

hipError_t launch_mg_solution(const MgGmres &G, int nact, double *out, int64_t ostride, hipStream_t st) {
    const int64_t n = G.Nd * G.K;
    if (nact <= 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(mg_solution_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nact), dim3(256), 0, st, G,
                       out, ostride);
    return hipGetLastError();
}

// rc(rhs) = in(rhs) rounded to FP32 (in: complex FP64 at in + rhs * istride).
__global__ void mg_load_kernel(MgGmres G, const double *in, int64_t istride) {
    const int64_t n = G.Nd * G.K;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int rhs = G.active[blockIdx.y];
    const double *x = in + (int64_t)rhs * istride + 2 * t;
    G.rc[(int64_t)rhs * G.vstride + t] = make_float2((float)x[0], (float)x[1]);
}

hipError_t launch_mg_load(const MgGmres &G, int nact, const double *in, int64_t istride, hipStream_t st) {
    const int64_t n = G.Nd * G.K;
    if (nact <= 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(mg_load_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nact), dim3(256), 0, st, G, in,
                       istride);
    return hipGetLastError();
}

}  // namespace sapdd
