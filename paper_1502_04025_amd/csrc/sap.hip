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
#include <cstdlib>
#include <cstring>

#include "blockgeo.hpp"
#include "kernels.hpp"

namespace sapdd {

template <class S, class SS, class P> struct SapArgs {  // S: links and clover, SS: spinors
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
    SS *rres;
    float *rres_sc;
    SS *delta;
    float *delta_sc;
    P *psi;
    int64_t psi_stride;  // elements per rhs
    const int *active;
    int nact;
    int64_t nblk;  // blocks of one colour
    int colour, mode, write_state, nmr;
};

// Sum of v over a full wave of 64 lanes in a fixed order, the same on every lane: DPP
// adds within each row of 16 lanes (lane ^ 1, lane ^ 2, then rotations by 4 and 8, after
// which every lane holds its row's sum), then the four rows' sums read from lanes 0, 16,
// 32 and 48. Register-to-register: no LDS round trip per step as with __shfl_xor.
template <int CTRL> __device__ __forceinline__ float dpp_add(float v) {
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF,
                                                                     false));
}
__device__ __forceinline__ float lane_value(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ float wave64_sum(float v) {
    v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x124>(v);  // row_ror:4
    v = dpp_add<0x128>(v);  // row_ror:8
    return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

// Sum three values over the workgroup in a fixed order; every thread gets the sums.
template <class BK, class R>
__device__ __forceinline__ void block_sum3(R &a, R &b, R &c, R *red) {
    if constexpr (BK::W == 64 && sizeof(R) == 4) {
        a = wave64_sum(a);
        b = wave64_sum(b);
        c = wave64_sum(c);
    } else {
#pragma unroll
        for (int off = BK::W / 2; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, BK::W);
            b += __shfl_xor(b, off, BK::W);
            c += __shfl_xor(c, off, BK::W);
        }
    }
    // the waves' sums of one value side by side (red is 16-byte aligned), so that every
    // thread reads them with a few wide loads, all issued before the first add
    constexpr int NW = BK::NW;
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[wv] = a;
        red[NW + wv] = b;
        red[2 * NW + wv] = c;
    }
    __syncthreads();
    R ra[NW], rb[NW], rc[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        ra[q] = red[q];
        rb[q] = red[NW + q];
        rc[q] = red[2 * NW + q];
    }
    a = ra[0];
    b = rb[0];
    c = rc[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
        a += ra[q];
        b += rb[q];
        c += rc[q];
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
template <int MU, class BK, class S, class SS, class P, class R, class LK>
__device__ __forceinline__ void gather_dir(const SapArgs<S, SS, P> &a, const SiteInfo &si, const LK &U,
                                           const int (&g)[4], const SS *dlt, const float *dlt_sc, R kappa,
                                           R (&rho)[24]) {
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

template <class BK, class S, class SS, class R, class P>
__global__ __launch_bounds__(BK::NT) __attribute__((amdgpu_waves_per_eu(SAPDD_SAP_WAVES_PER_EU)))
void sap_half_kernel(SapArgs<S, SS, P> a) {
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
    __shared__ __align__(16) R red[3 * BK::NW];
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

    SS *dlt = a.delta + (int64_t)rhs * V * 24;
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
    block_hop<BK, true, true>(1, si, U, T, H, lds);
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
        block_hop<BK, true, true>(0, si, U, A, H, lds);  // odd: H = H_oe r
        if (EARLY_AE && even) mul_even(A, T);  // even: T = A_e r (needs only r)
        if (!even) Xc.mul(H, T, (R)1);           // odd: T = A_o^-1 H_oe r
        // even: H = H_eo T; the reduction's barrier below separates these reads from the
        // next hop's writes, so a single-buffer hop needs no barrier of its own at the end
        block_hop<BK, false, true>(1, si, U, T, H, lds);
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
            const R inv = (R)1 / pp;  // one division for both parts
            ar = pr_re * inv;
            ai = pr_im * inv;
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
    block_hop<BK, true, true>(0, si, U, B, H, lds);
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

// ---------------------------------------------------------------------------- pair form
// The same half-sweep with one thread per pair of sites: thread s owns the even site and
// the odd site with half index s of its block, so a workgroup has Vbh threads and every
// wave works in both halves of a hop (it pushes from its site of the source parity, then
// pulls into its site of the other parity). A workgroup then needs half the waves and
// one hop buffer, and two (block, rhs) workgroups share a CU: while one waits at a
// barrier or on memory, the other issues. The split-parity kernel above leaves the odd
// waves idle while the even ones push and vice versa.
//
// The odd-site block residual rho_o, needed again at the end (delta_o = A_o^-1 (rho_o +
// kappa H_oe delta_e)), is parked in the thread's own delta slots, which nobody reads
// during this launch (the gather reads the other colour's corrections) and which the
// thread overwrites with its final delta: 24 values of the arithmetic type fit the two
// sites' slots in every storage precision, and no other thread touches them.
template <class BK> struct PairBlk {
    static constexpr int NT = BK::Vbh;
    static constexpr int W = NT < 64 ? NT : 64;
    static constexpr int NW = (NT + 63) / 64;
};

#ifndef SAPDD_SAP_LINK_AHEAD
#define SAPDD_SAP_LINK_AHEAD 1
#endif

template <class LK> struct LinkStorage;
template <class S, class R, bool C> struct LinkStorage<SiteLinks<S, R, C>> {
    typedef S type;
};

// The 16-byte vectors that hold link MU of a thread's site, loaded ahead of their use: a
// load issued after a barrier cannot be hoisted above it by the compiler, and the pull's
// first link would otherwise wait out its full cache latency right after the barrier.
template <int MU, class S> struct LinkAhead {
    typedef typename Vec<S>::type VT;
    static constexpr int W = Vec<S>::W, V0 = 18 * MU / W, V1 = (18 * MU + 17) / W, N = V1 - V0 + 1;
    VT x[N];
    template <class LK> __device__ __forceinline__ void load(const LK &U) {
        const VT *p = reinterpret_cast<const VT *>(U.base);
#pragma unroll
        for (int v = 0; v < N; ++v) x[v] = ld_vec<false>(p + vec_index<S, 72>(U.bp, V0 + v, U.s, U.Vbh));
    }
    template <class R> __device__ __forceinline__ void get(R out[18]) const {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const int q = 18 * MU + k - V0 * W;
            if constexpr (Storage<S>::scaled) out[k] = (R)(float)x[q / W][q % W];
            else out[k] = (R)x[q / W][q % W];
        }
    }
};

// pull_dir (branch-free) with the link of direction MU given.
template <int MU, class BK, class R, class LK, class LA>
__device__ __forceinline__ void pull_dir_ahead(const SiteInfo &si, const LK &U, const LA &la, R (&out)[24],
                                               const R *__restrict__ sp, const R *__restrict__ hb) {
    constexpr int Vbh = BK::Vbh;
    const bool f = (si.fin >> MU) & 1u, b = (si.bin >> MU) & 1u;
    {
        R chi[24], h[12], uh[12], u[18];
        const int n = si.nbf[MU];
#pragma unroll
        for (int k = 0; k < 24; ++k) chi[k] = sp[k * Vbh + n];
        project<MU, -1>(chi, h);
        la.get(u);
        su3_mul(u, h, uh);
        accum_recon<MU, -1>(out, uh, f ? U.scale() : (R)0);
    }
    {
        R uh[12];
        const int n = si.nbb[MU];
#pragma unroll
        for (int k = 0; k < 12; ++k) uh[k] = hb[(MU * 12 + k) * Vbh + n];
        accum_recon<MU, +1>(out, uh, b ? (R)1 : (R)0);
    }
}

// In-block hop between the parities in pair form: this thread pushes `in` from its site
// of parity SRC and receives `out` at its site of the other parity. Both SAP kernels take
// the branch-free directions: they are bound by instruction issue, not by memory.
template <int SRC, class BK, bool TAIL = true, class R, class LK, int WANT>
__device__ __forceinline__ void pair_hop(const SiteInfo &se, const SiteInfo &so, const LK &Ue, const LK &Uo,
                                         const R (&in)[24], R (&out)[24], HopLds<BK, R, WANT> &lds) {
    constexpr int Vbh = BK::Vbh;
    R *__restrict__ sp = lds.sp();
    R *__restrict__ hb = lds.hb();
    const SiteInfo &ss = SRC == 0 ? se : so;
    const SiteInfo &sr = SRC == 0 ? so : se;
    const LK &Us = SRC == 0 ? Ue : Uo;
    const LK &Ur = SRC == 0 ? Uo : Ue;
#if SAPDD_SAP_LINK_AHEAD
    LinkAhead<0, typename LinkStorage<LK>::type> la;
    la.load(Ur);
#endif
#pragma unroll
    for (int k = 0; k < 24; ++k) sp[k * Vbh + ss.s] = in[k];
    push_dir<0, BK, true>(ss, Us, in, hb);
    push_dir<1, BK, true>(ss, Us, in, hb);
    push_dir<2, BK, true>(ss, Us, in, hb);
    push_dir<3, BK, true>(ss, Us, in, hb);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 24; ++k) out[k] = 0;
#if SAPDD_SAP_LINK_AHEAD
    pull_dir_ahead<0, BK>(sr, Ur, la, out, sp, hb);
#else
    pull_dir<0, BK, true>(sr, Ur, out, sp, hb);
#endif
    pull_dir<1, BK, true>(sr, Ur, out, sp, hb);
    pull_dir<2, BK, true>(sr, Ur, out, sp, hb);
    pull_dir<3, BK, true>(sr, Ur, out, sp, hb);
    if constexpr (HopLds<BK, R, WANT>::NBUF == 2) {
        lds.cur ^= 1;
    } else if constexpr (TAIL) {
        __syncthreads();
    }
}

// Park / fetch 24 values of type R in the 16-byte vectors of the thread's two delta slots
// (even site first), in a thread-private order.
template <class S, class R>
__device__ __forceinline__ void park(S *dlt, int64_t b, int s, int Vbh, const R (&v)[24]) {
    typedef typename Vec<S>::type VS;
    typedef R VR __attribute__((ext_vector_type(16 / sizeof(R))));
    constexpr int PER = 16 / sizeof(R);
    constexpr int NV = 24 / PER;           // vectors to park
    constexpr int NS = 24 / Vec<S>::W;     // vectors per site slot
    static_assert(NV <= 2 * NS, "two delta slots hold the parked spinor");
    VS *p = reinterpret_cast<VS *>(dlt);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        VR x;
#pragma unroll
        for (int w = 0; w < PER; ++w) x[w] = v[q * PER + w];
        const int site_p = q / NS, vv = q % NS;
        *gmem(reinterpret_cast<VR *>(p + vec_index<S, 24>(2 * b + site_p, vv, s, Vbh))) = x;
    }
}
template <class S, class R>
__device__ __forceinline__ void fetch(const S *dlt, int64_t b, int s, int Vbh, R (&v)[24]) {
    typedef typename Vec<S>::type VS;
    typedef R VR __attribute__((ext_vector_type(16 / sizeof(R))));
    constexpr int PER = 16 / sizeof(R);
    constexpr int NV = 24 / PER;
    constexpr int NS = 24 / Vec<S>::W;
    const VS *p = reinterpret_cast<const VS *>(dlt);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int site_p = q / NS, vv = q % NS;
        const VR x = *gmem(reinterpret_cast<const VR *>(p + vec_index<S, 24>(2 * b + site_p, vv, s, Vbh)));
#pragma unroll
        for (int w = 0; w < PER; ++w) v[q * PER + w] = x[w];
    }
}

#ifndef SAPDD_SAP_PAIR_WAVES_PER_EU
#define SAPDD_SAP_PAIR_WAVES_PER_EU 2
#endif

template <class BK, class S, class SS, class R, class P>
__global__ __launch_bounds__(PairBlk<BK>::NT) __attribute__((amdgpu_waves_per_eu(SAPDD_SAP_PAIR_WAVES_PER_EU)))
void sap_pair_kernel(SapArgs<S, SS, P> a) {
    constexpr int Vbh = BK::Vbh;
    typedef PairBlk<BK> PB;
    // one hop buffer: two workgroups per CU need their LDS to fit twice
    __shared__ R lds_hop[HopLds<BK, R, 1>::PER];
    __shared__ __align__(16) R red[3 * PB::NW];
    HopLds<BK, R, 1> lds{lds_hop, 0};

    const Geom &geo = a.geo;
    const int s = threadIdx.x;
    const SiteInfo se = site_info<BK>(s);
    const SiteInfo so = site_info<BK>(Vbh + s);
    // (block, rhs) numbering as in the split-parity kernel: the rhs of one block follow
    // each other on one XCD, so its links and clover come from that XCD's L2
    const int64_t w = blockIdx.x;
    const int64_t kq = w >> 3;
    const int slot = (int)(kq % a.nact);
    const int64_t kb = (kq / a.nact) * 8 + (w & 7);
    if (kb >= a.nblk) return;  // padding of the last group of 8 (uniform per workgroup)
    const int64_t b = colour_block(geo.G, a.colour, kb);
    const int rhs = a.active[slot];
    const R kappa = (R)a.kappa[rhs];
    const int64_t V = geo.V;

    SiteLinks<S, R, false> Ue, Uo;
    Ue.init(a.links, a.lscale, 2 * b, s, Vbh);
    Uo.init(a.links, a.lscale, 2 * b + 1, s, Vbh);
    SiteClover<S, R, false> Xe, Xo;  // X = kappa T (even: A_e = 1 + X), A_o^-1 - 1 (odd)
    const S *Xr = (const S *)a.X[rhs];
    const float *Xs = a.Xsc ? a.Xsc[rhs] : nullptr;
    Xe.init(Xr, Xs, 2 * b, s, Vbh);
    Xo.init(Xr, Xs, 2 * b + 1, s, Vbh);

    SS *dlt = a.delta + (int64_t)rhs * V * 24;
    float *dlt_sc = a.delta_sc ? a.delta_sc + (int64_t)rhs * V : nullptr;
    SS *rr = a.rres + (int64_t)rhs * V * 12;
    float *rr_sc = a.rres_sc ? a.rres_sc + (int64_t)rhs * (V / 2) : nullptr;

    // A: even rho, then the MR residual r; B: odd rho, then the MR solution x (even);
    // T, H: scratch
    R A[24], B[24], T[24], H[24];

    // ---- 1. block residual rho (even into A, odd into B)
    if (a.mode < 2) {
        const double *eta = a.eta + rhs * a.eta_stride;
        const double f = a.eta_scale ? a.eta_scale[(int64_t)rhs * a.eta_scale_stride] : 1.0;
        double e[24];
        load_site<double, 24>(eta, nullptr, 2 * b, s, Vbh, e);
#pragma unroll
        for (int k = 0; k < 24; ++k) A[k] = (R)(e[k] * f);
        load_site<double, 24>(eta, nullptr, 2 * b + 1, s, Vbh, e);
#pragma unroll
        for (int k = 0; k < 24; ++k) B[k] = (R)(e[k] * f);
    } else {
        load_site<R, 24>(rr, rr_sc, b, s, Vbh, A);
#pragma unroll
        for (int k = 0; k < 24; ++k) B[k] = 0;
    }
    if (a.mode >= 1) {
        int g[4];
        block_coords(geo.G, b, g);
        gather_dir<0, BK>(a, se, Ue, g, dlt, dlt_sc, kappa, A);
        gather_dir<1, BK>(a, se, Ue, g, dlt, dlt_sc, kappa, A);
        gather_dir<2, BK>(a, se, Ue, g, dlt, dlt_sc, kappa, A);
        gather_dir<3, BK>(a, se, Ue, g, dlt, dlt_sc, kappa, A);
        gather_dir<0, BK>(a, so, Uo, g, dlt, dlt_sc, kappa, B);
        gather_dir<1, BK>(a, so, Uo, g, dlt, dlt_sc, kappa, B);
        gather_dir<2, BK>(a, so, Uo, g, dlt, dlt_sc, kappa, B);
        gather_dir<3, BK>(a, so, Uo, g, dlt, dlt_sc, kappa, B);
    }
    // rho_o is needed again at the end: park it in this thread's delta slots
    park<SS, R>(dlt, b, s, Vbh, B);

    // ---- 2. bhat_e = rho_e + kappa H_eo A_o^-1 rho_o
    Xo.mul(B, T, (R)1);
    pair_hop<1, BK>(se, so, Ue, Uo, T, H, lds);
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        A[k] = fmac(kappa, H[k], A[k]);
        B[k] = 0;
    }

    // ---- 3. MR on Dhat = A_e - kappa^2 H_eo A_o^-1 H_oe
    const R k2 = kappa * kappa;
    for (int it = 0; it < a.nmr; ++it) {
        // odd: H = H_oe r, then T = A_o^-1 H. The hop's closing barrier comes after the
        // clover product (which touches no LDS), so a wave done with its pull goes on
        // to it instead of waiting, and its clover loads are not held behind a barrier.
        pair_hop<0, BK, false>(se, so, Ue, Uo, A, H, lds);
        Xo.mul(H, T, (R)1);
        __syncthreads();
        // even: H = H_eo T; the reduction's barrier below separates these reads from the
        // next hop's writes
        pair_hop<1, BK, false>(se, so, Ue, Uo, T, H, lds);
        Xe.mul(A, T, (R)1);  // even: T = A_e r, then p = T - kappa^2 H
        R pr_re = 0, pr_im = 0, pp = 0;
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
        block_sum3<PB>(pr_re, pr_im, pp, red);
        R ar = 0, ai = 0;
        if (pp > 0) {
            const R inv = (R)1 / pp;  // one division for both parts
            ar = pr_re * inv;
            ai = pr_im * inv;
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const R rr_ = A[2 * k], ri = A[2 * k + 1];
            const R qr = T[2 * k], qi = T[2 * k + 1];
            B[2 * k] = fmac(ar, rr_, fmac(-ai, ri, B[2 * k]));
            B[2 * k + 1] = fmac(ar, ri, fmac(ai, rr_, B[2 * k + 1]));
            A[2 * k] = fmac(-ar, qr, fmac(ai, qi, rr_));
            A[2 * k + 1] = fmac(-ar, qi, fmac(-ai, qr, ri));
        }
    }

    // ---- 4. delta: even B, odd A_o^-1 (rho_o + kappa H_oe delta_e)
    pair_hop<0, BK, false>(se, so, Ue, Uo, B, H, lds);  // the last use of LDS: no closing barrier
    fetch<SS, R>(dlt, b, s, Vbh, T);
#pragma unroll
    for (int k = 0; k < 24; ++k) T[k] = fmac(kappa, H[k], T[k]);
    Xo.mul(T, H, (R)1);  // H = delta_o

    // ---- 5. outputs: psi += delta, keep delta and the even-site residual
    P *ps = a.psi + rhs * a.psi_stride;
    if (a.mode == 2) {
        R old[24];
        load_site<R, 24>(ps, nullptr, 2 * b, s, Vbh, old);
#pragma unroll
        for (int k = 0; k < 24; ++k) old[k] += B[k];
        store_site<R, 24>(ps, nullptr, 2 * b, s, Vbh, old);
        load_site<R, 24>(ps, nullptr, 2 * b + 1, s, Vbh, old);
#pragma unroll
        for (int k = 0; k < 24; ++k) old[k] += H[k];
        store_site<R, 24>(ps, nullptr, 2 * b + 1, s, Vbh, old);
    } else {
        store_site<R, 24>(ps, nullptr, 2 * b, s, Vbh, B);
        store_site<R, 24>(ps, nullptr, 2 * b + 1, s, Vbh, H);
    }
    if (a.write_state) {
        store_site<R, 24>(dlt, dlt_sc, 2 * b, s, Vbh, B);
        store_site<R, 24>(dlt, dlt_sc, 2 * b + 1, s, Vbh, H);
        store_site<R, 24>(rr, rr_sc, b, s, Vbh, A);
    }
}

// Which form runs a half-sweep (both compute the same half-sweep, each in its own fixed
// order; both are checked against the oracle). The pair form needs two workgroups per CU to pay off, and its FP32-storage variants
// spill registers: measured on 48^3 x 96 (FP16 storage, 12 RHS, 124416 workgroups) it
// takes 23.5 ms per half-sweep against 29.3 ms, on 16^3 x 32 (FP32 storage, one RHS, 128
// workgroups) 142 us against 73 us. So: the pair form for FP16 links and clover on
// lattices with at least one block of each colour per CU, the split-parity form otherwise
// (it also serves FP64 and 2^4 blocks). The choice depends on the geometry only, never on
// how many right-hand sides share the launch, so a right-hand side gets the same bits
// alone and in any batch. SAPDD_SAP_KERNEL=pair or =split in the environment forces one.
static int sap_form_override() {
    static const int v = [] {
        const char *e = getenv("SAPDD_SAP_KERNEL");
        if (e && strcmp(e, "split") == 0) return 1;
        if (e && strcmp(e, "pair") == 0) return 2;
        return 0;
    }();
    return v;
}
template <class S> static bool sap_pair_form(int64_t nblk) {
    const int o = sap_form_override();
    if (o) return o == 2;
    return Storage<S>::scaled && nblk >= 256;
}

template <class BK, class S, class SS, class R, class P>
static hipError_t sap_typed(const Geom &geo, const SapArgsHost &h, int colour, int mode, int ws, hipStream_t st) {
    SapArgs<S, SS, P> a;
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
    a.rres = (SS *)h.rres.data;
    a.rres_sc = h.rres.scale;
    a.delta = (SS *)h.delta.data;
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
    if constexpr (sizeof(R) == 4 && BK::Vbh >= 128) {
        if (sap_pair_form<S>(a.nblk)) {
            hipLaunchKernelGGL((sap_pair_kernel<BK, S, SS, R, P>), grid, dim3(PairBlk<BK>::NT), 0, st, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((sap_half_kernel<BK, S, SS, R, P>), grid, dim3(BK::NT), 0, st, a);
    return hipGetLastError();
}

// Storage combinations: (links and clover, Schwarz spinors, output psi). FP16 links and
// clover with FP32 spinors is the paper's half-precision mode (Sec. 3.3); FP16 spinors as
// well halve the spinor traffic; FP64 output serves the preconditioned vectors of
// deflated restarts.
template <class BK>
static hipError_t sap_shape(const Geom &geo, const SapArgsHost &h, int colour, int mode, int ws, hipStream_t st) {
    const int lp = h.links.prec, sp = h.rres.prec, pp = h.psi_prec;
    if (h.delta.prec != sp) return hipErrorInvalidValue;
    if (lp == P64 && sp == P64 && pp == P64)
        return sap_typed<BK, double, double, double, double>(geo, h, colour, mode, ws, st);
    if (lp == P32 && sp == P32 && pp == P32) return sap_typed<BK, float, float, float, float>(geo, h, colour, mode, ws, st);
    if (lp == P16 && sp == P16 && pp == P32)
        return sap_typed<BK, half_t, half_t, float, float>(geo, h, colour, mode, ws, st);
    if (lp == P16 && sp == P32 && pp == P32)
        return sap_typed<BK, half_t, float, float, float>(geo, h, colour, mode, ws, st);
    if (lp == P32 && sp == P32 && pp == P64)
        return sap_typed<BK, float, float, float, double>(geo, h, colour, mode, ws, st);
    if (lp == P16 && sp == P16 && pp == P64)
        return sap_typed<BK, half_t, half_t, float, double>(geo, h, colour, mode, ws, st);
    if (lp == P16 && sp == P32 && pp == P64)
        return sap_typed<BK, half_t, float, float, double>(geo, h, colour, mode, ws, st);
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
