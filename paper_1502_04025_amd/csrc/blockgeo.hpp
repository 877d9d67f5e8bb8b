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

// The four forward links of a thread's own site, either held in registers (in storage
// precision, converted on use) or re-read from global memory on every use.
template <class S, class R, bool CACHE> struct SiteLinks;

template <class S, class R> struct SiteLinks<S, R, true> {
    S u[72];
    R sc;
    __device__ __forceinline__ void init(const S *__restrict__ base, const float *__restrict__ scale,
                                         int64_t bp, int s, int Vbh) {
        const S *p = base + bp * 72 * (int64_t)Vbh + s;
#pragma unroll
        for (int k = 0; k < 72; ++k) u[k] = p[(int64_t)k * Vbh];
        if constexpr (Storage<S>::scaled) sc = (R)scale[bp * Vbh + s];
        else sc = (R)1;
    }
    template <int MU> __device__ __forceinline__ void get(R out[18]) const {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            if constexpr (Storage<S>::scaled) out[k] = (R)(float)u[18 * MU + k] * sc;
            else out[k] = (R)u[18 * MU + k];
        }
    }
};

template <class S, class R> struct SiteLinks<S, R, false> {
    const S *p;
    R sc;
    int Vbh;
    __device__ __forceinline__ void init(const S *__restrict__ base, const float *__restrict__ scale,
                                         int64_t bp, int s, int vbh) {
        Vbh = vbh;
        p = base + bp * 72 * (int64_t)Vbh + s;
        if constexpr (Storage<S>::scaled) sc = (R)scale[bp * Vbh + s];
        else sc = (R)1;
    }
    template <int MU> __device__ __forceinline__ void get(R out[18]) const {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            if constexpr (Storage<S>::scaled) out[k] = (R)(float)p[(int64_t)(18 * MU + k) * Vbh] * sc;
            else out[k] = (R)p[(int64_t)(18 * MU + k) * Vbh];
        }
    }
};

// Per-site packed clover (72 reals), held or re-read like the links.
template <class S, class R, bool CACHE> struct SiteClover;

template <class S, class R> struct SiteClover<S, R, true> {
    S x[72];
    R sc;
    __device__ __forceinline__ void init(const S *__restrict__ base, const float *__restrict__ scale,
                                         int64_t bp, int s, int Vbh) {
        const S *p = base + bp * 72 * (int64_t)Vbh + s;
#pragma unroll
        for (int k = 0; k < 72; ++k) x[k] = p[(int64_t)k * Vbh];
        if constexpr (Storage<S>::scaled) sc = (R)scale[bp * Vbh + s];
        else sc = (R)1;
    }
    __device__ __forceinline__ void get(R out[72]) const {
#pragma unroll
        for (int k = 0; k < 72; ++k) {
            if constexpr (Storage<S>::scaled) out[k] = (R)(float)x[k] * sc;
            else out[k] = (R)x[k];
        }
    }
};

template <class S, class R> struct SiteClover<S, R, false> {
    const S *p;
    R sc;
    int Vbh;
    __device__ __forceinline__ void init(const S *__restrict__ base, const float *__restrict__ scale,
                                         int64_t bp, int s, int vbh) {
        Vbh = vbh;
        p = base + bp * 72 * (int64_t)Vbh + s;
        if constexpr (Storage<S>::scaled) sc = (R)scale[bp * Vbh + s];
        else sc = (R)1;
    }
    __device__ __forceinline__ void get(R out[72]) const {
#pragma unroll
        for (int k = 0; k < 72; ++k) {
            if constexpr (Storage<S>::scaled) out[k] = (R)(float)p[(int64_t)k * Vbh] * sc;
            else out[k] = (R)p[(int64_t)k * Vbh];
        }
    }
};

// In-block hopping term between the two parities, via LDS.
//   Threads of parity `src` supply `in`. Threads of the other parity receive
//   out = sum_mu [ (1 - gamma_mu) U_mu(x) in(x + mu) + (1 + gamma_mu) U_mu(x - mu)^+ in(x - mu) ]
//   over the neighbours inside the block (hops leaving the block are dropped).
// Source threads store their spinor (for the forward hops of their backward neighbours)
// and, for every in-block forward neighbour, the transported half spinor
// U_mu(x)^+ (1 + gamma_mu) in(x); the receiving threads then need only their own links.
// Every thread of the workgroup must call this; it contains two barriers.
template <class BK, class R, class LK>
__device__ __forceinline__ void block_hop(int src, const SiteInfo &si, const LK &U, const R in[24], R out[24],
                                          R *__restrict__ sp, R *__restrict__ hb) {
    constexpr int Vbh = BK::Vbh;
    if (si.p == src) {
#pragma unroll
        for (int k = 0; k < 24; ++k) sp[k * Vbh + si.s] = in[k];
        static_for<0, 4>([&](auto m) {
            constexpr int MU = decltype(m)::value;
            if (si.fin & (1u << MU)) {
                R h[12], uh[12], u[18];
                project<MU, +1>(in, h);
                U.template get<MU>(u);
                su3_dag_mul(u, h, uh);
#pragma unroll
                for (int k = 0; k < 12; ++k) hb[(MU * 12 + k) * Vbh + si.s] = uh[k];
            }
        });
    }
    __syncthreads();
    if (si.p != src) {
#pragma unroll
        for (int k = 0; k < 24; ++k) out[k] = 0;
        static_for<0, 4>([&](auto m) {
            constexpr int MU = decltype(m)::value;
            if (si.fin & (1u << MU)) {
                R chi[24], h[12], uh[12], u[18];
                const int n = si.nbf[MU];
#pragma unroll
                for (int k = 0; k < 24; ++k) chi[k] = sp[k * Vbh + n];
                project<MU, -1>(chi, h);
                U.template get<MU>(u);
                su3_mul(u, h, uh);
                accum_recon<MU, -1>(out, uh, (R)1);
            }
            if (si.bin & (1u << MU)) {
                R uh[12];
                const int n = si.nbb[MU];
#pragma unroll
                for (int k = 0; k < 12; ++k) uh[k] = hb[(MU * 12 + k) * Vbh + n];
                accum_recon<MU, +1>(out, uh, (R)1);
            }
        });
    }
    __syncthreads();
}

}  // namespace sapdd
