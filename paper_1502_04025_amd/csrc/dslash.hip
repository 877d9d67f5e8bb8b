// dslash.hip - the Wilson-clover operator M on the whole lattice and its block-diagonal
// part M_B (the domain-internal operator of the Schwarz splitting, Sec. 3.1).
//
// Full operator: one thread per (site, right-hand side); neighbours are read straight
// from global memory. Workgroups are numbered so that the nact right-hand sides of one
// chunk of sites run back to back on the same XCD (workgroup w runs on XCD w mod 8), so
// links and clover of the chunk are re-read from that XCD's L2 rather than from HBM, and
// so that the chunks of one block share an XCD too.
//
// Block operator: one workgroup per (block, rhs), the block's spinor staged in LDS and
// the hops through the block faces masked off.
#include "blockgeo.hpp"
#include "kernels.hpp"

namespace sapdd {

template <class T> struct CF {  // typed const field view
    const T *data;
    const float *scale;
};
template <class T> struct MF {
    T *data;
    float *scale;
};

template <class BK> struct GeoC {  // geometry with compile-time block extents
    static __device__ __forceinline__ void site(const Geom &geo, const int x[4], int64_t &bp, int &s) {
        const int B[4] = {BK::bx, BK::by, BK::bz, BK::bt};
        int g[4], l[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            g[mu] = x[mu] / B[mu];
            l[mu] = x[mu] - g[mu] * B[mu];
        }
        bp = block_index(geo.G, g) * 2 + ((l[0] + l[1] + l[2] + l[3]) & 1);
        s = local_half_index(B, l);
    }
    static __device__ __forceinline__ void coords(const Geom &geo, int64_t bp, int s, int x[4]) {
        const int B[4] = {BK::bx, BK::by, BK::bz, BK::bt};
        int g[4], l[4];
        block_coords(geo.G, bp >> 1, g);
        local_coords(B, (int)(bp & 1), s, l);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) x[mu] = g[mu] * B[mu] + l[mu];
    }
};

constexpr int DSLASH_WG = 256;

// Chunks of DSLASH_WG sites that make up one block (its even half, then its odd half):
// they go to the same XCD, so the hops between the two halves, most of a site's
// neighbours, find the other half in that XCD's L2.
template <class BK> constexpr int full_chunks_per_block() {
    return 2 * BK::Vbh > DSLASH_WG ? 2 * BK::Vbh / DSLASH_WG : 1;
}



template <class BK, class S, class TI, class TO, class R>
__global__ __launch_bounds__(DSLASH_WG) void dslash_full_kernel(Geom geo, CF<S> links, CF<S> tclov, R kappa,
                                                                 CF<TI> in, MF<TO> out, const double *sub,
                                                                 double *part, const int *active, int nact,
                                                                 int nchunk, int ins_, int outs_, int subs_,
                                                                 const double *kap) {
    constexpr int Vbh = BK::Vbh;
    constexpr int G = full_chunks_per_block<BK>();
    const int w = blockIdx.x;
    const int xcd = w & 7;
    const int k = w >> 3;
    const int slot = k % nact;
    const int q = k / nact;
    const int chunk = ((q / G) * 8 + xcd) * G + q % G;
    const int rhs = active ? active[slot] : slot;
    const int64_t site = (int64_t)chunk * DSLASH_WG + threadIdx.x;
    const bool valid = chunk < nchunk && site < geo.V;
    double nrm = 0.0;
    if (valid) {
        const int64_t bp = site / Vbh;
        const int s = (int)(site - bp * Vbh);
        int x[4];
        GeoC<BK>::coords(geo, bp, s, x);
        if (kap) kappa = (R)kap[rhs];
        const int64_t ioff = (int64_t)rhs * ins_ * geo.V * 24;
        const int64_t ooff = (int64_t)rhs * outs_ * geo.V * 24;
        const TI *ind = in.data + ioff;
        const float *ins = in.scale ? in.scale + (int64_t)rhs * ins_ * geo.V : nullptr;
        R acc[24];
#pragma unroll
        for (int c = 0; c < 24; ++c) acc[c] = 0;
        static_for<0, 4>([&](auto m) {
            constexpr int MU = decltype(m)::value;
            const int L = geo.L[MU];
            {  // forward hop: (1 - gamma) U_mu(x) psi(x + mu)
                int y[4] = {x[0], x[1], x[2], x[3]};
                R sg = 1;
                if (++y[MU] == L) {
                    y[MU] = 0;
                    if (MU == 3 && geo.antiperiodic) sg = -1;
                }
                int64_t nbp;
                int ns;
                GeoC<BK>::site(geo, y, nbp, ns);
                R chi[24], h[12], u[18], uh[12];
                load_site<R, 24>(ind, ins, nbp, ns, Vbh, chi);
                project<MU, -1>(chi, h);
                load_reals<R, 72, 18 * MU, 18, S, true>(links.data, nullptr, bp, s, Vbh, u);
                su3_mul(u, h, uh);
                accum_recon<MU, -1>(acc, uh, sg * site_scale<R, S>(links.scale, bp, s, Vbh));
            }
            {  // backward hop: (1 + gamma) U_mu(x - mu)^+ psi(x - mu)
                int y[4] = {x[0], x[1], x[2], x[3]};
                R sg = 1;
                if (--y[MU] < 0) {
                    y[MU] = L - 1;
                    if (MU == 3 && geo.antiperiodic) sg = -1;
                }
                int64_t nbp;
                int ns;
                GeoC<BK>::site(geo, y, nbp, ns);
                R chi[24], h[12], u[18], uh[12];
                load_site<R, 24>(ind, ins, nbp, ns, Vbh, chi);
                project<MU, +1>(chi, h);
                load_reals<R, 72, 18 * MU, 18, S, true>(links.data, nullptr, nbp, ns, Vbh, u);
                su3_dag_mul(u, h, uh);
                accum_recon<MU, +1>(acc, uh, sg * site_scale<R, S>(links.scale, nbp, ns, Vbh));
            }
        });
        R psi[24], res[24];
        load_site<R, 24>(ind, ins, bp, s, Vbh, psi);
        CloverRegs<S, R> cl;
        cl.load(tclov.data, tclov.scale, bp, s, Vbh);
        clover_mul(cl, psi, res, kappa);  // (1 + kappa T) psi
#pragma unroll
        for (int c = 0; c < 24; ++c) res[c] = fmac(-kappa, acc[c], res[c]);
        if (sub) {
            double sb[24];
            load_site<double, 24>(sub + (int64_t)rhs * subs_ * geo.V * 24, nullptr, bp, s, Vbh, sb);
#pragma unroll
            for (int c = 0; c < 24; ++c) res[c] = (R)sb[c] - res[c];
        }
        store_site<R, 24>(out.data + ooff, out.scale ? out.scale + (int64_t)rhs * outs_ * geo.V : nullptr, bp, s, Vbh,
                          res);
        if (part) {
#pragma unroll
            for (int c = 0; c < 24; ++c) nrm += (double)res[c] * (double)res[c];
        }
    }
    if (part) {  // fixed-order workgroup reduction of |out|^2
        __shared__ double red[DSLASH_WG / 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0;
            for (int q = 0; q < DSLASH_WG / 64; ++q) t += red[q];
            const int nwg = (nchunk + 7) / 8 * 8;
            if (chunk < nwg) part[(int64_t)slot * nwg + chunk] = t;
        }
    }
}

int dslash_full_partials(const Geom &geo) {
    const int nchunk = (int)((geo.V + DSLASH_WG - 1) / DSLASH_WG);
    return (nchunk + 7) / 8 * 8;
}

template <class BK, class S, class TI, class TO, class R>
static hipError_t full_typed(const Geom &geo, Fld links, Fld tclov, double kappa, const DslashIO &io,
                             hipStream_t st) {
    const int nchunk = (int)((geo.V + DSLASH_WG - 1) / DSLASH_WG);
    constexpr int G = full_chunks_per_block<BK>();
    // groups of G chunks dealt round-robin to the 8 XCDs; every chunk index below
    // dslash_full_partials gets a workgroup (those past the lattice write zero partials)
    const int ng8 = ((nchunk + G - 1) / G + 7) / 8 * 8;
    const int64_t nwg = (int64_t)ng8 * G * io.nact;
    if (nwg == 0) return hipSuccess;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((dslash_full_kernel<BK, S, TI, TO, R>), dim3((unsigned)nwg), dim3(DSLASH_WG), 0, st, geo,
                       CF<S>{(const S *)links.data, links.scale}, CF<S>{(const S *)tclov.data, tclov.scale},
                       (R)kappa, CF<TI>{(const TI *)io.in.data, io.in.scale}, MF<TO>{(TO *)io.out.data, io.out.scale},
                       io.sub, io.part, io.active, io.nact, nchunk, io.in_stride, io.out_stride, io.sub_stride,
                       io.kappa);
    return hipGetLastError();
}

template <class BK>
static hipError_t full_shape(const Geom &geo, Fld links, Fld tclov, double kappa, const DslashIO &io,
                             hipStream_t st) {
    // supported combinations: FP64 links with FP64 or FP32 input and FP64 output (the
    // outer solver), and uniform FP32 / FP16 storage (the operator API).
    if (links.prec == P64) {
        if (io.out.prec != P64) return hipErrorInvalidValue;
        if (io.in.prec == P64) return full_typed<BK, double, double, double, double>(geo, links, tclov, kappa, io, st);
        if (io.in.prec == P32) return full_typed<BK, double, float, double, double>(geo, links, tclov, kappa, io, st);
        return hipErrorInvalidValue;
    }
    if (io.sub) return hipErrorInvalidValue;
    if (links.prec == P32 && io.in.prec == P32 && io.out.prec == P32)
        return full_typed<BK, float, float, float, float>(geo, links, tclov, kappa, io, st);
    if (links.prec == P16 && io.in.prec == P16 && io.out.prec == P16)
        return full_typed<BK, half_t, half_t, half_t, float>(geo, links, tclov, kappa, io, st);
    return hipErrorInvalidValue;
}

// Call F<Blk<...>>(args...) for the supported block shapes.
template <template <class> class F, class... A>
static hipError_t by_shape(const Geom &geo, A &&...args) {
    if (geo.B[0] == 2 && geo.B[1] == 2 && geo.B[2] == 2 && geo.B[3] == 2) return F<Blk<2, 2, 2, 2>>::run(args...);
    if (geo.B[0] == 4 && geo.B[1] == 4 && geo.B[2] == 4 && geo.B[3] == 4) return F<Blk<4, 4, 4, 4>>::run(args...);
    if (geo.B[0] == 8 && geo.B[1] == 4 && geo.B[2] == 4 && geo.B[3] == 4) return F<Blk<8, 4, 4, 4>>::run(args...);
    return hipErrorInvalidValue;
}

template <class BK> struct FullRun {
    static hipError_t run(const Geom &geo, Fld links, Fld tclov, double kappa, const DslashIO &io, hipStream_t st) {
        return full_shape<BK>(geo, links, tclov, kappa, io, st);
    }
};

hipError_t launch_dslash_full(const Geom &geo, Fld links, Fld tclov, double kappa, const DslashIO &io,
                              hipStream_t st) {
    return by_shape<FullRun>(geo, geo, links, tclov, kappa, io, st);
}

// ---------------------------------------------------------------- block operator
template <class BK, class S, class R>
__global__ __launch_bounds__(BK::NT) void dslash_block_kernel(Geom geo, CF<S> links, CF<S> tclov, R kappa,
                                                               CF<S> in, MF<S> out) {
    constexpr int Vbh = BK::Vbh;
    // one LDS buffer: this memory-bound kernel gains more from occupancy than from the
    // barrier a second buffer would save
    __shared__ R lds_hop[HopLds<BK, R, 1>::PER];
    HopLds<BK, R, 1> lds{lds_hop, 0};
    const SiteInfo si = site_info<BK>(threadIdx.x);
    const int64_t b = blockIdx.x;
    const int rhs = blockIdx.y;
    const int64_t bp = 2 * b + si.p;
    const int64_t ioff = (int64_t)rhs * geo.V * 24, soff = (int64_t)rhs * geo.V;
    // links held in registers between the two half-hops (re-reading them from L1/L2 to
    // reach 4 waves per SIMD measured slower: 3.65 vs 4.53 TB/s in FP16)
    // Every byte this kernel touches is used by one workgroup only: non-temporal hints
    // (measured 4.71 -> 5.52 TB/s in FP32, 4.49 -> 4.80 TB/s in FP16 on 32^3x64). Issuing
    // the clover loads before the hops instead of after measured slower.
    constexpr bool NT = true;
    SiteLinks<S, R, true> U;
    U.template init<NT>(links.data, links.scale, bp, si.s, Vbh);
    R psi[24], hop[24];
    load_site<R, 24, S, NT>(in.data + ioff, in.scale ? in.scale + soff : nullptr, bp, si.s, Vbh, psi);
    block_hop<BK>(0, si, U, psi, hop, lds);  // odd sites receive
    block_hop<BK>(1, si, U, psi, hop, lds);  // even sites receive
    R res[24];
    CloverRegs<S, R> cl;
    cl.template load<NT>(tclov.data, tclov.scale, bp, si.s, Vbh);
    clover_mul(cl, psi, res, kappa);
#pragma unroll
    for (int c = 0; c < 24; ++c) res[c] = fmac(-kappa, hop[c], res[c]);
    store_site<R, 24, S, NT>(out.data + ioff, out.scale ? out.scale + soff : nullptr, bp, si.s, Vbh, res);
}

template <class BK>
static hipError_t block_shape(const Geom &geo, Fld links, Fld tclov, double kappa, Fld in, Fld out, int nrhs,
                              hipStream_t st) {
    if (links.prec != in.prec || in.prec != out.prec || tclov.prec != links.prec) return hipErrorInvalidValue;
    dim3 grid((unsigned)geo.Nd, (unsigned)nrhs);
    if (links.prec == P64)
        hipLaunchKernelGGL((dslash_block_kernel<BK, double, double>), grid, dim3(BK::NT), 0, st, geo,
                           CF<double>{(const double *)links.data, nullptr}, CF<double>{(const double *)tclov.data, nullptr},
                           kappa, CF<double>{(const double *)in.data, nullptr}, MF<double>{(double *)out.data, nullptr});
    else if (links.prec == P32)
        hipLaunchKernelGGL((dslash_block_kernel<BK, float, float>), grid, dim3(BK::NT), 0, st, geo,
                           CF<float>{(const float *)links.data, nullptr}, CF<float>{(const float *)tclov.data, nullptr},
                           (float)kappa, CF<float>{(const float *)in.data, nullptr}, MF<float>{(float *)out.data, nullptr});
    else
        hipLaunchKernelGGL((dslash_block_kernel<BK, half_t, float>), grid, dim3(BK::NT), 0, st, geo,
                           CF<half_t>{(const half_t *)links.data, links.scale},
                           CF<half_t>{(const half_t *)tclov.data, tclov.scale}, (float)kappa,
                           CF<half_t>{(const half_t *)in.data, in.scale}, MF<half_t>{(half_t *)out.data, out.scale});
    return hipGetLastError();
}

template <class BK> struct BlockRun {
    static hipError_t run(const Geom &geo, Fld links, Fld tclov, double kappa, Fld in, Fld out, int nrhs,
                          hipStream_t st) {
        return block_shape<BK>(geo, links, tclov, kappa, in, out, nrhs, st);
    }
};

hipError_t launch_dslash_block(const Geom &geo, Fld links, Fld tclov, double kappa, Fld in, Fld out, int nrhs,
                               hipStream_t st) {
    if (nrhs <= 0 || geo.Nd == 0) return hipSuccess;
    return by_shape<BlockRun>(geo, geo, links, tclov, kappa, in, out, nrhs, st);
}

}  // namespace sapdd
