// blockgeo.hpp - compile-time Schwarz block shapes, per-thread site information inside a
// block, and the in-block hopping term evaluated through LDS.
//
// One workgroup owns one block (the GPU counterpart of the paper's one-domain-per-core
// assignment, Sec. 3.3/3.5); thread tid < Vbh is the even site with half index tid and
// thread Vbh + s the odd site s, so the two parities occupy separate waves whenever
// Vbh >= 64.
#pragma once
#include <utility>

#include "core.hpp"

namespace sapdd {

template <int I, int N, class F> __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

template <int BX, int BY, int BZ, int BT> struct Blk {
    static constexpr int bx = BX, by = BY, bz = BZ, bt = BT;
    static constexpr int Vb = BX * BY * BZ * BT;
    static constexpr int Vbh = Vb / 2;
    static constexpr int NT = Vb;                         // threads per workgroup
    static constexpr int W = NT < 64 ? NT : 64;           // lanes used per wave
    static constexpr int NW = (NT + 63) / 64;             // waves per workgroup
    __device__ static constexpr int ext(int mu) { return mu == 0 ? BX : mu == 1 ? BY : mu == 2 ? BZ : BT; }
};

struct SiteInfo {
    int p, s;
    int l[4];
    int nbf[4], nbb[4];  // half index of the in-block forward / backward neighbour
    unsigned fin, bin;   // bit mu set if that neighbour is inside the block
};

template <class BK> __device__ __forceinline__ SiteInfo site_info(int tid) {
    SiteInfo si;
    si.p = tid >= BK::Vbh;
    si.s = tid - si.p * BK::Vbh;
    const int B[4] = {BK::bx, BK::by, BK::bz, BK::bt};
    local_coords(B, si.p, si.s, si.l);
    si.fin = si.bin = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        int lf[4] = {si.l[0], si.l[1], si.l[2], si.l[3]};
        int lb[4] = {si.l[0], si.l[1], si.l[2], si.l[3]};
        lf[mu] += 1;
        lb[mu] -= 1;
        si.nbf[mu] = si.nbb[mu] = 0;
        if (si.l[mu] < B[mu] - 1) {
            si.fin |= 1u << mu;
            si.nbf[mu] = local_half_index(B, lf);
        }
        if (si.l[mu] > 0) {
            si.bin |= 1u << mu;
            si.nbb[mu] = local_half_index(B, lb);
        }
    }
    return si;
}

// The four forward links of a thread's own site, either held in registers (as the
// storage-precision 16-byte vectors they were loaded in, converted on use) or re-read
// from global memory on every use.
template <class S, class R, bool CACHE> struct SiteLinks;

template <class S, class R> struct SiteLinks<S, R, true> {
    typedef typename Vec<S>::type VT;
    static constexpr int W = Vec<S>::W;
    VT u[72 / W];
    R sc;
    template <bool NT = false>
    __device__ __forceinline__ void init(const S *__restrict__ base, const float *__restrict__ scale,
                                         int64_t bp, int s, int Vbh) {
        const VT *p = reinterpret_cast<const VT *>(base);
#pragma unroll
        for (int v = 0; v < 72 / W; ++v) u[v] = ld_vec<NT>(p + vec_index<S, 72>(bp, v, s, Vbh));
        if constexpr (Storage<S>::scaled) sc = (R)*gmem(scale + bp * Vbh + s);
        else sc = (R)1;
    }
    // Link MU without the FP16 site scale (see scale()).
    template <int MU> __device__ __forceinline__ void get(R out[18]) const {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const int q = 18 * MU + k;
            if constexpr (Storage<S>::scaled) out[k] = (R)(float)u[q / W][q % W];
            else out[k] = (R)u[q / W][q % W];
        }
    }
    __device__ __forceinline__ R scale() const {
        if constexpr (Storage<S>::scaled) return sc;
        else return (R)1;
    }
};

template <class S, class R> struct SiteLinks<S, R, false> {
    const S *base;
    R sc;
    int64_t bp;
    int s, Vbh;
    __device__ __forceinline__ void init(const S *__restrict__ b, const float *__restrict__ scl, int64_t bp_, int s_,
                                         int vbh) {
        base = b;
        bp = bp_;
        s = s_;
        Vbh = vbh;
        sc = site_scale<R, S>(scl, bp, s, Vbh);
    }
    // Link MU without the FP16 site scale (see scale()).
    template <int MU> __device__ __forceinline__ void get(R out[18]) const {
        load_reals<R, 72, 18 * MU, 18, S, true>(base, nullptr, bp, s, Vbh, out);
    }
    __device__ __forceinline__ R scale() const {
        if constexpr (Storage<S>::scaled) return sc;
        else return (R)1;
    }
};

// Per-site packed clover (72 reals) in registers as the storage-precision vectors it was
// loaded in; entries are converted one at a time where they are used.
template <class S, class R> struct CloverRegs {
    typedef typename Vec<S>::type VT;
    static constexpr int W = Vec<S>::W;
    VT x[72 / W];
    R sc;
    template <bool NT = false>
    __device__ __forceinline__ void load(const S *__restrict__ base, const float *__restrict__ scale, int64_t bp,
                                         int s, int Vbh) {
        const VT *p = reinterpret_cast<const VT *>(base);
#pragma unroll
        for (int v = 0; v < 72 / W; ++v) x[v] = ld_vec<NT>(p + vec_index<S, 72>(bp, v, s, Vbh));
        if constexpr (Storage<S>::scaled) sc = (R)*gmem(scale + bp * Vbh + s);
        else sc = (R)1;
    }
    // Entry k without the FP16 site scale (clover_mul applies it).
    __device__ __forceinline__ R at(int k) const {
        if constexpr (Storage<S>::scaled) return (R)(float)x[k / W][k % W];
        else return (R)x[k / W][k % W];
    }
    __device__ __forceinline__ R scale() const {
        if constexpr (Storage<S>::scaled) return sc;
        else return (R)1;
    }
};

// out = in + kx * X in for the two packed Hermitian 6x6 blocks of X: X in is accumulated
// from the stored entries with FMAs and scaled once (kx times the site scale).
template <class XR, class R>
__device__ __forceinline__ void clover_mul(const XR &X, const R (&in)[24], R (&out)[24], R kx) {
    const R f = kx * X.scale();
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const int o = 12 * blk;
        R t[12];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const R d = X.at(36 * blk + i);
            t[2 * i] = fmac(d, in[o + 2 * i], (R)0);
            t[2 * i + 1] = fmac(d, in[o + 2 * i + 1], (R)0);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j) {
                const int q = 36 * blk + 6 + 2 * (i * 5 - i * (i - 1) / 2 + (j - i - 1));
                const R xr = X.at(q), xi = X.at(q + 1);
                t[2 * i] = fmac(xr, in[o + 2 * j], t[2 * i]);
                t[2 * i] = fmac(-xi, in[o + 2 * j + 1], t[2 * i]);
                t[2 * i + 1] = fmac(xr, in[o + 2 * j + 1], t[2 * i + 1]);
                t[2 * i + 1] = fmac(xi, in[o + 2 * j], t[2 * i + 1]);
                t[2 * j] = fmac(xr, in[o + 2 * i], t[2 * j]);
                t[2 * j] = fmac(xi, in[o + 2 * i + 1], t[2 * j]);
                t[2 * j + 1] = fmac(xr, in[o + 2 * i + 1], t[2 * j + 1]);
                t[2 * j + 1] = fmac(-xi, in[o + 2 * i], t[2 * j + 1]);
            }
#pragma unroll
        for (int k = 0; k < 12; ++k) out[o + k] = fmac(f, t[k], in[o + k]);
    }
}

// The clover of a thread's own site, held in registers for the whole kernel or re-read
// (from the L1/L2 caches) at every use.
template <class S, class R, bool CACHE> struct SiteClover;

template <class S, class R> struct SiteClover<S, R, true> {
    CloverRegs<S, R> c;
    __device__ __forceinline__ void init(const S *__restrict__ base, const float *__restrict__ scale, int64_t bp,
                                         int s, int Vbh) {
        c.load(base, scale, bp, s, Vbh);
    }
    __device__ __forceinline__ void mul(const R (&in)[24], R (&out)[24], R kx) const { clover_mul(c, in, out, kx); }
};

template <class S, class R> struct SiteClover<S, R, false> {
    const S *base;
    const float *scale;
    int64_t bp;
    int s, Vbh;
    __device__ __forceinline__ void init(const S *__restrict__ b, const float *__restrict__ sc, int64_t bp_, int s_,
                                         int vbh) {
        base = b;
        scale = sc;
        bp = bp_;
        s = s_;
        Vbh = vbh;
    }
    __device__ __forceinline__ void mul(const R (&in)[24], R (&out)[24], R kx) const {
        CloverRegs<S, R> c;
        c.load(base, scale, bp, s, Vbh);
        clover_mul(c, in, out, kx);
    }
};

// In-block hopping term between the two parities, via LDS.
//   Threads of parity `src` supply `in`. Threads of the other parity receive
//   out = sum_mu [ (1 - gamma_mu) U_mu(x) in(x + mu) + (1 + gamma_mu) U_mu(x - mu)^+ in(x - mu) ]
//   over the neighbours inside the block (hops leaving the block are dropped); source
//   threads leave `out` untouched.
// Source threads store their spinor (for the forward hops of their backward neighbours)
// and, for every in-block forward neighbour, the transported half spinor
// U_mu(x)^+ (1 + gamma_mu) in(x); the receiving threads then need only their own links.
// Every thread of the workgroup must call this; it contains one barrier (two with a
// single LDS buffer).
//
// BF (branch-free): every lane does the work of every direction. The face conditions
// differ between the lanes of a wave, so a branch issues the work for the whole wave
// anyway; without it the compiler schedules the four directions as one stream. Lanes
// without the in-block forward neighbour write a slot nobody reads, and receivers without
// the neighbour accumulate it with weight zero; every slot a receiver reads has been
// written, so the zero weights only ever meet finite values. This loads the links of the
// face sites too, which the operator does not need: the instruction-bound SAP kernels
// use it, the memory-bound block operator does not.
template <int MU, class BK, bool BF, class R, class LK>
__device__ __forceinline__ void push_dir(const SiteInfo &si, const LK &U, const R (&in)[24], R *__restrict__ hb) {
    constexpr int Vbh = BK::Vbh;
    if (BF || (si.fin & (1u << MU))) {
        R h[12], uh[12], u[18];
        project<MU, +1>(in, h);
        U.template get<MU>(u);
        su3_dag_mul(u, h, uh);
        const R sc = U.scale();
#pragma unroll
        for (int k = 0; k < 12; ++k) hb[(MU * 12 + k) * Vbh + si.s] = sc * uh[k];
    }
}

template <int MU, class BK, bool BF, class R, class LK>
__device__ __forceinline__ void pull_dir(const SiteInfo &si, const LK &U, R (&out)[24], const R *__restrict__ sp,
                                         const R *__restrict__ hb) {
    constexpr int Vbh = BK::Vbh;
    const bool f = (si.fin >> MU) & 1u, b = (si.bin >> MU) & 1u;
    if (BF || f) {
        R chi[24], h[12], uh[12], u[18];
        const int n = si.nbf[MU];
#pragma unroll
        for (int k = 0; k < 24; ++k) chi[k] = sp[k * Vbh + n];
        project<MU, -1>(chi, h);
        U.template get<MU>(u);
        su3_mul(u, h, uh);
        accum_recon<MU, -1>(out, uh, f ? U.scale() : (R)0);
    }
    if (BF || b) {
        R uh[12];
        const int n = si.nbb[MU];
#pragma unroll
        for (int k = 0; k < 12; ++k) uh[k] = hb[(MU * 12 + k) * Vbh + n];
        accum_recon<MU, +1>(out, uh, b ? (R)1 : (R)0);
    }
}

// LDS exchange area of block_hop: NBUF buffers of (spinor + 4 transported half
// spinors) per source site. With two buffers consecutive hops alternate between them
// and each hop needs only its middle barrier: a thread can only start writing buffer i
// again (hop n + 2) after passing hop n + 1's barrier, which every thread reaches only
// after finishing its reads of hop n.
template <class BK, class R, int WANT = 2> struct HopLds {
    static constexpr int PER = 72 * BK::Vbh;  // reals per buffer: 24 (spinor) + 48 (half spinors)
    static constexpr int NBUF = WANT == 2 && 2 * PER * (int)sizeof(R) <= 150 * 1024 ? 2 : 1;
    R *base;
    int cur;
    __device__ __forceinline__ R *sp() const { return base + cur * PER; }
    __device__ __forceinline__ R *hb() const { return base + cur * PER + 24 * BK::Vbh; }
};

// TAIL = false (one LDS buffer only): the caller guarantees a barrier between the
// receivers' reads and the next hop's writes, and the trailing barrier is left out.
template <class BK, bool TAIL = true, bool BF = false, class R, class LK, int WANT>
__device__ __forceinline__ void block_hop(int src, const SiteInfo &si, const LK &U, const R (&in)[24], R (&out)[24],
                                          HopLds<BK, R, WANT> &lds) {
    constexpr int Vbh = BK::Vbh;
    R *__restrict__ sp = lds.sp();
    R *__restrict__ hb = lds.hb();
    if (si.p == src) {
#pragma unroll
        for (int k = 0; k < 24; ++k) sp[k * Vbh + si.s] = in[k];
        push_dir<0, BK, BF>(si, U, in, hb);
        push_dir<1, BK, BF>(si, U, in, hb);
        push_dir<2, BK, BF>(si, U, in, hb);
        push_dir<3, BK, BF>(si, U, in, hb);
    }
    __syncthreads();
    if (si.p != src) {
#pragma unroll
        for (int k = 0; k < 24; ++k) out[k] = 0;
        pull_dir<0, BK, BF>(si, U, out, sp, hb);
        pull_dir<1, BK, BF>(si, U, out, sp, hb);
        pull_dir<2, BK, BF>(si, U, out, sp, hb);
        pull_dir<3, BK, BF>(si, U, out, sp, hb);
    }
    if constexpr (HopLds<BK, R, WANT>::NBUF == 2) {
        lds.cur ^= 1;
    } else if constexpr (TAIL) {
        __syncthreads();  // one buffer: the next hop may only overwrite it after every read
    }
}

}  // namespace sapdd
