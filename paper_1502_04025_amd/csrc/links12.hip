// links12.hip - the block-diagonal operator M_B with every link stored as its first two
// rows (12 reals per direction instead of 18). The third row of a special unitary 3x3
// matrix is the complex conjugate of the cross product of the first two, so each link is
// rebuilt where it is used; the in-block operator then reads a third fewer link bytes.
// Hops inside a block never cross the antiperiodic time boundary (blocks never wrap), so
// no boundary sign has to be kept beside the links. The links must be special unitary,
// which a gauge field is; the library does not check it.
//
// Storage: 48 reals per site, real k = 12 mu + 2 (3 row + col) + (0 re, 1 im) for rows
// 0 and 1, in the block-tiled layout of every other field (FP32, or FP16 with one FP32
// scale per site over the 48 reals).
#include "blockgeo.hpp"
#include "kernels.hpp"

namespace sapdd {

namespace {

template <class S, class R> struct SiteLinks12 {
    typedef typename Vec<S>::type VT;
    static constexpr int W = Vec<S>::W;
    VT u[48 / W];
    R sc;
    template <bool NT = false>
    __device__ __forceinline__ void init(const S *__restrict__ base, const float *__restrict__ scale, int64_t bp, int s,
                                         int Vbh) {
        const VT *p = reinterpret_cast<const VT *>(base);
#pragma unroll
        for (int v = 0; v < 48 / W; ++v) u[v] = ld_vec<NT>(p + vec_index<S, 48>(bp, v, s, Vbh));
        if constexpr (Storage<S>::scaled) sc = (R)scale[bp * Vbh + s];
        else sc = (R)1;
    }
    __device__ __forceinline__ R raw(int q) const {
        if constexpr (Storage<S>::scaled) return (R)(float)u[q / W][q % W];
        else return (R)u[q / W][q % W];
    }
    // Link MU without the FP16 site scale, as the 18-real accessors give it. Rows 0 and 1
    // come from storage; row 2 = conj(row 0 x row 1). Stored rows carry 1 / sc each, so
    // the product carries 1 / sc^2 and is multiplied by sc once.
    template <int MU> __device__ __forceinline__ void get(R out[18]) const {
#pragma unroll
        for (int k = 0; k < 12; ++k) out[k] = raw(12 * MU + k);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const R a1r = out[2 * c1], a1i = out[2 * c1 + 1], a2r = out[2 * c2], a2i = out[2 * c2 + 1];
            const R b1r = out[6 + 2 * c1], b1i = out[6 + 2 * c1 + 1], b2r = out[6 + 2 * c2], b2i = out[6 + 2 * c2 + 1];
            const R pr = (a1r * b2r - a1i * b2i) - (a2r * b1r - a2i * b1i);
            const R pi = (a1r * b2i + a1i * b2r) - (a2r * b1i + a2i * b1r);
            out[12 + 2 * c] = pr * sc;
            out[12 + 2 * c + 1] = -pi * sc;
        }
    }
    __device__ __forceinline__ R scale() const {
        if constexpr (Storage<S>::scaled) return sc;
        else return (R)1;
    }
};

// Rows 0 and 1 of every link of the FP64 block-tiled field, in storage type S.
template <class S>
__global__ void links12_pack_kernel(Geom geo, const double *__restrict__ links, S *__restrict__ out,
                                    float *__restrict__ scale) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= geo.V) return;
    const int s = (int)(t % geo.Vbh);
    const int64_t bp = t / geo.Vbh;
    double all[72];
    load_site<double, 72, double>(links, nullptr, bp, s, geo.Vbh, all);
    float v[48];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int k = 0; k < 12; ++k) v[12 * mu + k] = (float)all[18 * mu + k];
    store_site<float, 48, S>(out, scale, bp, s, geo.Vbh, v);
}

template <class BK, class S, class R>
__global__ __launch_bounds__(BK::NT) void dslash_block12_kernel(Geom geo, const S *links12, const float *lscale,
                                                                const S *tclov, const float *tscale, R kappa,
                                                                const S *in, const float *inscale, S *out,
                                                                float *outscale) {
    constexpr int Vbh = BK::Vbh;
    __shared__ R lds_hop[HopLds<BK, R, 1>::PER];
    HopLds<BK, R, 1> lds{lds_hop, 0};
    const SiteInfo si = site_info<BK>(threadIdx.x);
    const int64_t b = blockIdx.x;
    const int rhs = blockIdx.y;
    const int64_t bp = 2 * b + si.p;
    const int64_t ioff = (int64_t)rhs * geo.V * 24, soff = (int64_t)rhs * geo.V;
    constexpr bool NT = true;  // every byte is used by one workgroup only
    SiteLinks12<S, R> U;
    U.template init<NT>(links12, lscale, bp, si.s, Vbh);
    R psi[24], hop[24];
    load_site<R, 24, S, NT>(in + ioff, inscale ? inscale + soff : nullptr, bp, si.s, Vbh, psi);
    block_hop<BK>(0, si, U, psi, hop, lds);  // odd sites receive
    block_hop<BK>(1, si, U, psi, hop, lds);  // even sites receive
    R res[24];
    CloverRegs<S, R> cl;
    cl.template load<NT>(tclov, tscale, bp, si.s, Vbh);
    clover_mul(cl, psi, res, kappa);
#pragma unroll
    for (int c = 0; c < 24; ++c) res[c] = fmac(-kappa, hop[c], res[c]);
    store_site<R, 24, S, NT>(out + ioff, outscale ? outscale + soff : nullptr, bp, si.s, Vbh, res);
}

template <class BK>
hipError_t block12_shape(const Geom &geo, Fld links12, Fld tclov, double kappa, Fld in, Fld out, int nrhs,
                         hipStream_t st) {
    if (links12.prec != in.prec || in.prec != out.prec || tclov.prec != links12.prec) return hipErrorInvalidValue;
    const dim3 grid((unsigned)geo.Nd, (unsigned)nrhs);
    if (links12.prec == P32)
        hipLaunchKernelGGL((dslash_block12_kernel<BK, float, float>), grid, dim3(BK::NT), 0, st, geo,
                           (const float *)links12.data, nullptr, (const float *)tclov.data, nullptr, (float)kappa,
                           (const float *)in.data, nullptr, (float *)out.data, nullptr);
    else if (links12.prec == P16)
        hipLaunchKernelGGL((dslash_block12_kernel<BK, half_t, float>), grid, dim3(BK::NT), 0, st, geo,
                           (const half_t *)links12.data, links12.scale, (const half_t *)tclov.data, tclov.scale,
                           (float)kappa, (const half_t *)in.data, in.scale, (half_t *)out.data, out.scale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_links12_pack(const Geom &geo, const double *links64, Fld out, hipStream_t st) {
    if (geo.V == 0) return hipSuccess;
    const unsigned nb = (unsigned)((geo.V + 255) / 256);
    if (out.prec == P32)
        hipLaunchKernelGGL(links12_pack_kernel<float>, dim3(nb), dim3(256), 0, st, geo, links64, (float *)out.data,
                           nullptr);
    else if (out.prec == P16)
        hipLaunchKernelGGL(links12_pack_kernel<half_t>, dim3(nb), dim3(256), 0, st, geo, links64,
                           (half_t *)out.data, out.scale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_dslash_block12(const Geom &geo, Fld links12, Fld tclov, double kappa, Fld in, Fld out, int nrhs,
                                 hipStream_t st) {
    if (nrhs <= 0 || geo.Nd == 0) return hipSuccess;
    if (geo.B[0] == 2 && geo.B[1] == 2 && geo.B[2] == 2 && geo.B[3] == 2)
        return block12_shape<Blk<2, 2, 2, 2>>(geo, links12, tclov, kappa, in, out, nrhs, st);
    if (geo.B[0] == 4 && geo.B[1] == 4 && geo.B[2] == 4 && geo.B[3] == 4)
        return block12_shape<Blk<4, 4, 4, 4>>(geo, links12, tclov, kappa, in, out, nrhs, st);
    if (geo.B[0] == 8 && geo.B[1] == 4 && geo.B[2] == 4 && geo.B[3] == 4)
        return block12_shape<Blk<8, 4, 4, 4>>(geo, links12, tclov, kappa, in, out, nrhs, st);
    return hipErrorInvalidValue;
}

}  // namespace sapdd
