// sap.hip - one colour half-sweep of the Schwarz alternating procedure (Sec. 3.1): for
// every block B of one colour, in parallel, one workgroup
//   1. forms the block residual rho_B: the stored even-site MR residual of B's previous
//      solve (odd sites: 0), or the input eta on the first cycle, plus the change the
//      other colour's last corrections made to it - a gather of the hops from the
//      neighbouring blocks' corrections delta into B's boundary sites;
//   2. solves M_B delta = rho_B approximately with even-odd preconditioning:
//      bhat_e = rho_e - K_eo A_o^-1 rho_o, nmr minimal-residual steps on
//      Dhat = A_e - K_eo A_o^-1 K_oe from zero, delta_o = A_o^-1 (rho_o - K_oe delta_e),
//      with K = -kappa * (in-block hopping);
//   3. adds delta to psi and keeps delta and the new even-site residual for the next
//      half-sweep.
// The block never leaves the workgroup during the MR iterations: spinors live in
// registers and LDS, the in-block hops go through LDS (block_hop) and the MR inner
// products are wave-shuffle plus LDS reductions in a fixed order (so results do not
// depend on scheduling). Blocks of one colour share no site and no hop, so the gather
// form (each block reads its neighbours, nobody writes into another block) is race free.
//
// Clover input X per rhs: X = kappa T on even sites (A_e = 1 + X) and
// X = A_o^-1 - 1 on odd sites (A_o^-1 = 1 + X).
#include "blockgeo.hpp"
#include "kernels.hpp"

namespace sapdd {

template <class S, class P> struct SapArgs {
    Geom geo;
    const S *links;
    const float *lscale;
    const S *const *X;
    const float *const *Xsc;
    const double *kappa;
    const double *eta;
    const double *eta_scale;
    int eta_scale_stride;
    int64_t eta_stride;  // doubles per rhs
    S *rres;
    float *rres_sc;
    S *delta;
    float *delta_sc;
    P *psi;
    int64_t psi_stride;  // elements per rhs
    const int *active;
    int nact;
    int64_t nblk;  // blocks of one colour
    int colour, mode, write_state, nmr;
};

// Sum three values over the workgroup in a fixed order; every thread gets the sums.
template <class BK, class R>
__device__ __forceinline__ void block_sum3(R &a, R &b, R &c, R *red) {
#pragma unroll
    for (int off = BK::W / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, BK::W);
        b += __shfl_xor(b, off, BK::W);
        c += __shfl_xor(c, off, BK::W);
    }
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[3 * wv] = a;
        red[3 * wv + 1] = b;
        red[3 * wv + 2] = c;
    }
    __syncthreads();
    a = b = c = 0;
#pragma unroll
    for (int q = 0; q < BK::NW; ++q) {
        a += red[3 * q];
        b += red[3 * q + 1];
        c += red[3 * q + 2];
    }
}

// Register policy: whether a thread keeps its links / clover in registers for the whole
// block solve (re-reading them from the L1/L2 caches otherwise).
#ifndef SAPDD_SAP_CACHE_LINKS
#define SAPDD_SAP_CACHE_LINKS 0
#endif
#ifndef SAPDD_SAP_CACHE_CLOVER
#define SAPDD_SAP_CACHE_CLOVER 0
#endif

#ifndef SAPDD_SAP_XLDS
#define SAPDD_SAP_XLDS 1
#endif

// The clover of a thread's own site held in LDS (thread-private slots k * Vbh + s).
template <class S, class R, int Vbh> struct LdsClover {
    const S *x;
    int s;
    R sc;
    __device__ __forceinline__ R at(int k) const {
        if constexpr (Storage<S>::scaled) return (R)(float)x[k * Vbh + s];
        else return (R)x[k * Vbh + s];
    }
    __device__ __forceinline__ R scale() const { return sc; }
};

#ifndef SAPDD_SAP_WAVES_PER_EU
#define SAPDD_SAP_WAVES_PER_EU 2
#endif

// Hops into site x across its block faces in direction mu, from the neighbouring blocks'
// corrections delta: rho += kappa * [ (1 - gamma) U_mu(x) delta(x + mu) on the forward
// face, (1 + gamma) U_mu(x - mu)^+ delta(x - mu) on the backward face ].
template <int MU, class BK, class S, class P, class R, class LK>
__device__ __forceinline__ void gather_dir(const SapArgs<S, P> &a, const SiteInfo &si, const LK &U, const int (&g)[4],
                                           const S *dlt, const float *dlt_sc, R kappa, R (&rho)[24]) {
    constexpr int Vbh = BK::Vbh;
    const Geom &geo = a.geo;
    const int B[4] = {BK::bx, BK::by, BK::bz, BK::bt};
    if (!(si.fin & (1u << MU))) {  // x + mu lies in the next block
        int gn[4] = {g[0], g[1], g[2], g[3]}, ln[4] = {si.l[0], si.l[1], si.l[2], si.l[3]};
        R sg = 1;
        if (++gn[MU] == geo.G[MU]) {
            gn[MU] = 0;
            if (MU == 3 && geo.antiperiodic) sg = -1;
        }
        ln[MU] = 0;
        const int64_t nbp = 2 * block_index(geo.G, gn) + (1 - si.p);
        const int ns = local_half_index(B, ln);
        R d[24], h[12], u[18], uh[12];
        load_site<R, 24>(dlt, dlt_sc, nbp, ns, Vbh, d);
        project<MU, -1>(d, h);
        U.template get<MU>(u);
        su3_mul(u, h, uh);
        accum_recon<MU, -1>(rho, uh, kappa * sg * U.scale());
    }
    if (!(si.bin & (1u << MU))) {  // x - mu lies in the previous block
        int gn[4] = {g[0], g[1], g[2], g[3]}, ln[4] = {si.l[0], si.l[1], si.l[2], si.l[3]};
        R sg = 1;
        if (--gn[MU] < 0) {
            gn[MU] = geo.G[MU] - 1;
            if (MU == 3 && geo.antiperiodic) sg = -1;
        }
        ln[MU] = B[MU] - 1;
        const int64_t nbp = 2 * block_index(geo.G, gn) + (1 - si.p);
        const int ns = local_half_index(B, ln);
        R d[24], h[12], u[18], uh[12];
        load_site<R, 24>(dlt, dlt_sc, nbp, ns, Vbh, d);
        load_reals<R, 72, 18 * MU, 18, S, true>(a.links, nullptr, nbp, ns, Vbh, u);
        const R lsc = site_scale<R, S>(a.lscale, nbp, ns, Vbh);
        project<MU, +1>(d, h);
        su3_dag_mul(u, h, uh);
        accum_recon<MU, +1>(rho, uh, kappa * sg * lsc);
    }
}

template <class BK, class S, class R, class P>
__global__ __launch_bounds__(BK::NT) __attribute__((amdgpu_waves_per_eu(SAPDD_SAP_WAVES_PER_EU)))
void sap_half_kernel(SapArgs<S, P> a) {
    constexpr int Vbh = BK::Vbh;
    constexpr bool CACHE_L = sizeof(R) == 4 && SAPDD_SAP_CACHE_LINKS;
    constexpr bool CACHE_X = sizeof(R) == 4 && SAPDD_SAP_CACHE_CLOVER;
    // FP16 storage: even sites form A_e r during the odd sites' half of the MR step
    // (4^4 blocks, 12 RHS: 425 -> 403 us per half-sweep). With FP32 or FP64 storage the
    // extra live spinor across the hop costs more registers than the overlap gains
    // (8x4^3 FP32: 84 -> 127 us), so A_e r is formed after the hop there.
    constexpr bool EARLY_AE = Storage<S>::scaled;
    // XL: on 8x4x4x4 blocks the even sites' clover is copied into LDS once and read from
    // there in every MR step, and the hop uses one LDS buffer. With FP32 storage the links
    // and clover of the 16 blocks an XCD works on at once exceed its 4 MB L2 otherwise
    // (16^3x32, 1 RHS: 83.7 -> 74.6 us per half-sweep). Links in LDS, or the odd sites'
    // clover as well (FP16), measured slower.
    constexpr bool XL = SAPDD_SAP_XLDS && sizeof(R) == 4 && BK::Vbh == 256;
    constexpr int HB = XL ? 1 : 2;
    __shared__ R lds_hop[HopLds<BK, R, HB>::NBUF * HopLds<BK, R, HB>::PER];
    __shared__ S xl[XL ? 72 * Vbh : 1];
    __shared__ R red[3 * BK::NW];
    HopLds<BK, R, HB> lds{lds_hop, 0};

    const Geom &geo = a.geo;
    const SiteInfo si = site_info<BK>(threadIdx.x);
    // Workgroup w runs on XCD w mod 8. Number the (block, rhs) pairs so that the nact
    // right-hand sides of one block follow each other on the same XCD: the block's links
    // and clover are then re-read from that XCD's L2 instead of HBM.
    const int64_t w = blockIdx.x;
    const int64_t kq = w >> 3;
    const int slot = (int)(kq % a.nact);
    const int64_t kb = (kq / a.nact) * 8 + (w & 7);
    if (kb >= a.nblk) return;  // padding of the last group of 8 (uniform per workgroup)
    const int64_t b = colour_block(geo.G, a.colour, kb);
    const int rhs = a.active[slot];
    const int64_t bp = 2 * b + si.p;
    const R kappa = (R)a.kappa[rhs];
    const int64_t V = geo.V;
    const bool even = si.p == 0;

    SiteLinks<S, R, CACHE_L> U;
    U.init(a.links, a.lscale, bp, si.s, Vbh);
    SiteClover<S, R, CACHE_X> Xc;
    Xc.init(a.X[rhs], a.Xsc ? a.Xsc[rhs] : nullptr, bp, si.s, Vbh);
    LdsClover<S, R, Vbh> Xe{xl, si.s, (R)1};
    if (XL && even) {
        CloverRegs<S, R> c;
        c.load(a.X[rhs], a.Xsc ? a.Xsc[rhs] : nullptr, bp, si.s, Vbh);
        constexpr int W = Vec<S>::W;
#pragma unroll
        for (int v = 0; v < 72 / W; ++v)
#pragma unroll
            for (int q = 0; q < W; ++q) xl[(v * W + q) * Vbh + si.s] = c.x[v][q];
        Xe.sc = c.scale();
    }
    // even sites: T = (1 + X) in
    auto mul_even = [&](const R(&in)[24], R(&out)[24]) {
        if constexpr (XL) clover_mul(Xe, in, out, (R)1);
        else Xc.mul(in, out, (R)1);
    };

    S *dlt = a.delta + (int64_t)rhs * V * 24;
    float *dlt_sc = a.delta_sc ? a.delta_sc + (int64_t)rhs * V : nullptr;

    // Per-thread spinors. Even sites: A = MR residual r, B = MR solution; odd sites:
    // A = block residual rho_o. T and H are scratch (H receives the in-block hops).
    R A[24], B[24], T[24], H[24];

    // ---- 1. block residual rho into A
    if (a.mode < 2) {
        double e[24];
        load_site<double, 24>(a.eta + rhs * a.eta_stride, nullptr, bp, si.s, Vbh, e);
        const double f = a.eta_scale ? a.eta_scale[(int64_t)rhs * a.eta_scale_stride] : 1.0;
#pragma unroll
        for (int k = 0; k < 24; ++k) A[k] = (R)(e[k] * f);
    } else if (even) {
        load_site<R, 24>(a.rres + (int64_t)rhs * V * 12, a.rres_sc ? a.rres_sc + (int64_t)rhs * (V / 2) : nullptr, b,
                         si.s, Vbh, A);
    } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) A[k] = 0;
    }
    if (a.mode >= 1) {
        // rho(x) -= sum_y M_{x,y} delta(y) over hops from neighbouring blocks: M = -kappa * hop there.
        int g[4];
        block_coords(geo.G, b, g);
        gather_dir<0, BK>(a, si, U, g, dlt, dlt_sc, kappa, A);
        gather_dir<1, BK>(a, si, U, g, dlt, dlt_sc, kappa, A);
        gather_dir<2, BK>(a, si, U, g, dlt, dlt_sc, kappa, A);
        gather_dir<3, BK>(a, si, U, g, dlt, dlt_sc, kappa, A);
    }

    // ---- 2. bhat_e = rho_e + kappa H_eo A_o^-1 rho_o (odd: T = A_o^-1 rho_o)
    if (!even) Xc.mul(A, T, (R)1);
    block_hop<BK>(1, si, U, T, H, lds);
    if (even) {
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            A[k] = fmac(kappa, H[k], A[k]);
            B[k] = 0;
        }
    }

    // ---- 3. MR on Dhat = A_e - kappa^2 H_eo A_o^-1 H_oe
    const R k2 = kappa * kappa;
    for (int it = 0; it < a.nmr; ++it) {
        block_hop<BK>(0, si, U, A, H, lds);  // odd: H = H_oe r
        if (EARLY_AE && even) mul_even(A, T);  // even: T = A_e r (needs only r)
        if (!even) Xc.mul(H, T, (R)1);           // odd: T = A_o^-1 H_oe r
        // even: H = H_eo T; the reduction's barrier below separates these reads from the
        // next hop's writes, so a single-buffer hop needs no barrier of its own at the end
        block_hop<BK, false>(1, si, U, T, H, lds);
        R pr_re = 0, pr_im = 0, pp = 0;
        if (even) {
            if (!EARLY_AE) mul_even(A, T);  // even: T = p = A_e r - kappa^2 H
#pragma unroll
            for (int k = 0; k < 24; ++k) T[k] = fmac(-k2, H[k], T[k]);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                pr_re = fmac(T[2 * k], A[2 * k], pr_re);
                pr_re = fmac(T[2 * k + 1], A[2 * k + 1], pr_re);
                pr_im = fmac(T[2 * k], A[2 * k + 1], pr_im);
                pr_im = fmac(-T[2 * k + 1], A[2 * k], pr_im);
                pp = fmac(T[2 * k], T[2 * k], pp);
                pp = fmac(T[2 * k + 1], T[2 * k + 1], pp);
            }
        }
        block_sum3<BK>(pr_re, pr_im, pp, red);
        R ar = 0, ai = 0;
        if (pp > 0) {
            ar = pr_re / pp;
            ai = pr_im / pp;
        }
        if (even) {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const R rr = A[2 * k], ri = A[2 * k + 1];
                const R qr = T[2 * k], qi = T[2 * k + 1];
                B[2 * k] = fmac(ar, rr, fmac(-ai, ri, B[2 * k]));
                B[2 * k + 1] = fmac(ar, ri, fmac(ai, rr, B[2 * k + 1]));
                A[2 * k] = fmac(-ar, qr, fmac(ai, qi, rr));
                A[2 * k + 1] = fmac(-ar, qi, fmac(-ai, qr, ri));
            }
        }
    }

    // ---- 4. delta: even B, odd A_o^-1 (rho_o + kappa H_oe delta_e)
    block_hop<BK>(0, si, U, B, H, lds);
    if (!even) {
#pragma unroll
        for (int k = 0; k < 24; ++k) T[k] = fmac(kappa, H[k], A[k]);
        Xc.mul(T, B, (R)1);  // odd: B = delta_o
    }

    // ---- 5. outputs: psi += delta, keep delta and the even-site residual
    P *ps = a.psi + rhs * a.psi_stride;
    if (a.mode == 2) {
        R old[24];
        load_site<R, 24>(ps, nullptr, bp, si.s, Vbh, old);
#pragma unroll
        for (int k = 0; k < 24; ++k) old[k] += B[k];
        store_site<R, 24>(ps, nullptr, bp, si.s, Vbh, old);
    } else {
        store_site<R, 24>(ps, nullptr, bp, si.s, Vbh, B);
    }
    if (a.write_state) {
        store_site<R, 24>(dlt, dlt_sc, bp, si.s, Vbh, B);
        if (even)
            store_site<R, 24>(a.rres + (int64_t)rhs * V * 12, a.rres_sc ? a.rres_sc + (int64_t)rhs * (V / 2) : nullptr,
                              b, si.s, Vbh, A);
    }
}

template <class BK, class S, class R, class P>
static hipError_t sap_typed(const Geom &geo, const SapArgsHost &h, int colour, int mode, int ws, hipStream_t st) {
    SapArgs<S, P> a;
    a.geo = geo;
    a.links = (const S *)h.links.data;
    a.lscale = h.links.scale;
    a.X = (const S *const *)h.X;
    a.Xsc = h.Xsc;
    a.kappa = h.kappa;
    a.eta = h.eta;
    a.eta_scale = h.eta_scale;
    a.eta_scale_stride = h.eta_scale_stride;
    a.eta_stride = (int64_t)h.eta_stride_rhs * geo.V * 24;
    a.rres = (S *)h.rres.data;
    a.rres_sc = h.rres.scale;
    a.delta = (S *)h.delta.data;
    a.delta_sc = h.delta.scale;
    a.psi = (P *)h.psi;
    a.psi_stride = (int64_t)h.psi_stride_rhs * geo.V * 24;
    a.active = h.active;
    a.nact = h.nact;
    a.nblk = geo.Nd / 2;
    a.colour = colour;
    a.mode = mode;
    a.write_state = ws;
    a.nmr = h.nmr;
    const int64_t nwg = (geo.Nd / 2 + 7) / 8 * 8 * h.nact;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid((unsigned)nwg);
    hipLaunchKernelGGL((sap_half_kernel<BK, S, R, P>), grid, dim3(BK::NT), 0, st, a);
    return hipGetLastError();
}

template <class BK>
static hipError_t sap_shape(const Geom &geo, const SapArgsHost &h, int colour, int mode, int ws, hipStream_t st) {
    const int sp = h.links.prec;
    if (sp == P64 && h.psi_prec == P64) return sap_typed<BK, double, double, double>(geo, h, colour, mode, ws, st);
    if (sp == P32 && h.psi_prec == P32) return sap_typed<BK, float, float, float>(geo, h, colour, mode, ws, st);
    if (sp == P16 && h.psi_prec == P32) return sap_typed<BK, half_t, float, float>(geo, h, colour, mode, ws, st);
    // FP64 output: the preconditioned vectors of deflated restarts
    if (sp == P32 && h.psi_prec == P64) return sap_typed<BK, float, float, double>(geo, h, colour, mode, ws, st);
    if (sp == P16 && h.psi_prec == P64) return sap_typed<BK, half_t, float, double>(geo, h, colour, mode, ws, st);
    return hipErrorInvalidValue;
}

hipError_t launch_sap_half(const Geom &geo, const SapArgsHost &a, int colour, int mode, int write_state,
                           hipStream_t st) {
    if (a.nact <= 0) return hipSuccess;
    if (geo.B[0] == 2 && geo.B[1] == 2 && geo.B[2] == 2 && geo.B[3] == 2)
        return sap_shape<Blk<2, 2, 2, 2>>(geo, a, colour, mode, write_state, st);
    if (geo.B[0] == 4 && geo.B[1] == 4 && geo.B[2] == 4 && geo.B[3] == 4)
        return sap_shape<Blk<4, 4, 4, 4>>(geo, a, colour, mode, write_state, st);
    if (geo.B[0] == 8 && geo.B[1] == 4 && geo.B[2] == 4 && geo.B[3] == 4)
        return sap_shape<Blk<8, 4, 4, 4>>(geo, a, colour, mode, write_state, st);
    return hipErrorInvalidValue;
}

}  // namespace sapdd
