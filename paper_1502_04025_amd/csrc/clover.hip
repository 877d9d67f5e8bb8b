// clover.hip - the Sheikholeslami-Wohlert clover term of the Wilson-clover operator
// (Sec. 3.1) and the per-site matrices the Schwarz sweep needs.
//
// T(x) = -c_sw sum_{mu<nu} gamma_mu gamma_nu (x) F_mu,nu(x), F = (Q - Q^+)/8 minus its
// trace / 3, Q = sum of the four plaquettes in the (mu, nu) plane that start and end at
// x, all traversed mu-then-nu. In the chiral basis gamma_mu gamma_nu is block diagonal:
// G_mu G_nu^+ on spins 0-1 and G_mu^+ G_nu on spins 2-3, so T is two 6x6 Hermitian
// blocks (72 reals, packed as described in core.hpp). All of it is FP64 and one-time
// per gauge field (T) or per kappa (the inverse).
#include "core.hpp"
#include "kernels.hpp"

namespace sapdd {

constexpr int CLOVER_WG = 128;

struct Cx {
    double r, i;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ Cx cconj(Cx a) { return {a.r, -a.i}; }

struct M3 {
    Cx e[3][3];
};

__device__ __forceinline__ M3 mmul(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const Cx p = cmul(a.e[i][k], b.e[k][j]);
                s.r += p.r;
                s.i += p.i;
            }
            c.e[i][j] = s;
        }
    return c;
}

__device__ __forceinline__ M3 mdag(const M3 &a) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.e[i][j] = cconj(a.e[j][i]);
    return c;
}

// U_mu at global coordinates x (periodic wrap), from the block-tiled FP64 links.
__device__ M3 link_at(const Geom &geo, const double *links, const int xin[4], int mu) {
    int x[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) x[d] = ((xin[d] % geo.L[d]) + geo.L[d]) % geo.L[d];
    int64_t bp;
    int s;
    site_of(geo, x, bp, s);
    M3 u;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            u.e[a][b].r = links[real_index<double, 72>(bp, 18 * mu + 2 * (3 * a + b), s, geo.Vbh)];
            u.e[a][b].i = links[real_index<double, 72>(bp, 18 * mu + 2 * (3 * a + b) + 1, s, geo.Vbh)];
        }
    return u;
}

// Chiral-block factor of gamma_mu: G[mu][row][col] (DeGrand-Rossi basis).
__device__ __forceinline__ Cx gmat(int mu, int r, int c) {
    // G_x = [[0, i], [i, 0]], G_y = [[0, -1], [1, 0]], G_z = [[i, 0], [0, -i]], G_t = 1
    switch (mu) {
    case 0: return r != c ? Cx{0, 1} : Cx{0, 0};
    case 1: return r != c ? (r == 0 ? Cx{-1, 0} : Cx{1, 0}) : Cx{0, 0};
    case 2: return r == c ? (r == 0 ? Cx{0, 1} : Cx{0, -1}) : Cx{0, 0};
    default: return r == c ? Cx{1, 0} : Cx{0, 0};
    }
}

// 2x2 spin factor of gamma_mu gamma_nu on chiral block k: G_mu G_nu^+ (k = 0), G_mu^+ G_nu (k = 1).
__device__ __forceinline__ Cx spin_factor(int k, int mu, int nu, int s, int t) {
    Cx acc = {0, 0};
    for (int q = 0; q < 2; ++q) {
        Cx p;
        if (k == 0) p = cmul(gmat(mu, s, q), cconj(gmat(nu, t, q)));
        else p = cmul(cconj(gmat(mu, q, s)), gmat(nu, q, t));
        acc.r += p.r;
        acc.i += p.i;
    }
    return acc;
}

__device__ __forceinline__ int upper_index(int a, int b) { return a * 5 - a * (a - 1) / 2 + (b - a - 1); }

// Pack a Hermitian 6x6 block (only the diagonal's real part and the upper triangle are kept).
__device__ __forceinline__ void pack6(const Cx m[6][6], double *out36) {
    for (int i = 0; i < 6; ++i) out36[i] = m[i][i].r;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j) {
            out36[6 + 2 * upper_index(i, j)] = m[i][j].r;
            out36[6 + 2 * upper_index(i, j) + 1] = m[i][j].i;
        }
}

__device__ __forceinline__ void unpack6(const double *in36, Cx m[6][6]) {
    for (int i = 0; i < 6; ++i) m[i][i] = {in36[i], 0.0};
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j) {
            const Cx v = {in36[6 + 2 * upper_index(i, j)], in36[6 + 2 * upper_index(i, j) + 1]};
            m[i][j] = v;
            m[j][i] = cconj(v);
        }
}

__global__ __launch_bounds__(CLOVER_WG) void clover_build_kernel(Geom geo, const double *links, double csw,
                                                                 double *tclov) {
    const int64_t t = (int64_t)blockIdx.x * CLOVER_WG + threadIdx.x;
    if (t >= geo.V) return;
    const int64_t bp = t / geo.Vbh;
    const int s = (int)(t - bp * geo.Vbh);
    int x[4];
    coords_of(geo, bp, s, x);
    Cx T[2][6][6];
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) T[k][i][j] = {0, 0};
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            int xm[4], xn[4], xmn[4], xmp[4], xpm[4], xmm[4], xpn[4];
            for (int d = 0; d < 4; ++d) xm[d] = xn[d] = xmn[d] = xmp[d] = xpm[d] = xmm[d] = xpn[d] = x[d];
            xpm[mu] += 1;                   // x + mu
            xpn[nu] += 1;                   // x + nu
            xm[mu] -= 1;                    // x - mu
            xn[nu] -= 1;                    // x - nu
            xmp[mu] -= 1; xmp[nu] += 1;     // x - mu + nu
            xmn[mu] += 1; xmn[nu] -= 1;     // x + mu - nu
            xmm[mu] -= 1; xmm[nu] -= 1;     // x - mu - nu
            const M3 um = link_at(geo, links, x, mu), un = link_at(geo, links, x, nu);
            // x -> x+mu -> x+mu+nu -> x+nu -> x
            M3 q = mmul(mmul(mmul(um, link_at(geo, links, xpm, nu)), mdag(link_at(geo, links, xpn, mu))), mdag(un));
            // x -> x+nu -> x+nu-mu -> x-mu -> x
            const M3 umm = link_at(geo, links, xm, mu);
            M3 l2 = mmul(mmul(mmul(un, mdag(link_at(geo, links, xmp, mu))), mdag(link_at(geo, links, xm, nu))), umm);
            // x -> x-mu -> x-mu-nu -> x-nu -> x
            const M3 unn = link_at(geo, links, xn, nu);
            M3 l3 = mmul(mmul(mmul(mdag(umm), mdag(link_at(geo, links, xmm, nu))), link_at(geo, links, xmm, mu)), unn);
            // x -> x-nu -> x-nu+mu -> x+mu -> x
            M3 l4 = mmul(mmul(mmul(mdag(unn), link_at(geo, links, xn, mu)), link_at(geo, links, xmn, nu)), mdag(um));
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    q.e[a][b].r += l2.e[a][b].r + l3.e[a][b].r + l4.e[a][b].r;
                    q.e[a][b].i += l2.e[a][b].i + l3.e[a][b].i + l4.e[a][b].i;
                }
            M3 f;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    f.e[a][b].r = (q.e[a][b].r - q.e[b][a].r) * 0.125;
                    f.e[a][b].i = (q.e[a][b].i + q.e[b][a].i) * 0.125;
                }
            const double tri = (f.e[0][0].i + f.e[1][1].i + f.e[2][2].i) / 3.0;  // trace is imaginary
            for (int a = 0; a < 3; ++a) f.e[a][a].i -= tri;
            for (int k = 0; k < 2; ++k)
                for (int sp = 0; sp < 2; ++sp)
                    for (int tp = 0; tp < 2; ++tp) {
                        const Cx g = spin_factor(k, mu, nu, sp, tp);
                        if (g.r == 0.0 && g.i == 0.0) continue;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) {
                                const Cx p = cmul(g, f.e[a][b]);
                                T[k][3 * sp + a][3 * tp + b].r -= csw * p.r;
                                T[k][3 * sp + a][3 * tp + b].i -= csw * p.i;
                            }
                    }
        }
    double packed[72];
    pack6(T[0], packed);
    pack6(T[1], packed + 36);
    store_site<double, 72>(tclov, nullptr, bp, s, geo.Vbh, packed);
}

__global__ __launch_bounds__(CLOVER_WG) void clover_pack_kernel(Geom geo, const double *canon, double *tclov) {
    const int64_t t = (int64_t)blockIdx.x * CLOVER_WG + threadIdx.x;
    if (t >= geo.V) return;
    const int64_t bp = t / geo.Vbh;
    const int s = (int)(t - bp * geo.Vbh);
    int x[4];
    coords_of(geo, bp, s, x);
    const int64_t ci = x[0] + (int64_t)geo.L[0] * (x[1] + (int64_t)geo.L[1] * (x[2] + (int64_t)geo.L[2] * x[3]));
    const double *src = canon + ci * 288;  // 12 x 12 complex
    double packed[72];
    for (int k = 0; k < 2; ++k) {
        Cx m[6][6];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                const int r = 6 * k + i, c = 6 * k + j;
                m[i][j] = {src[2 * (12 * r + c)], src[2 * (12 * r + c) + 1]};
            }
        pack6(m, packed + 36 * k);
    }
    store_site<double, 72>(tclov, nullptr, bp, s, geo.Vbh, packed);
}

// In-place Gauss-Jordan inverse with partial pivoting; returns false if a pivot
// magnitude falls below 1e-12.
__device__ bool invert6(Cx a[6][6], Cx inv[6][6]) {
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) inv[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    bool ok = true;
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        double best = a[c][c].r * a[c][c].r + a[c][c].i * a[c][c].i;
        for (int r = c + 1; r < 6; ++r) {
            const double m = a[r][c].r * a[r][c].r + a[r][c].i * a[r][c].i;
            if (m > best) { best = m; piv = r; }
        }
        if (!(best >= 1e-24)) { ok = false; best = 1e-24; }
        if (piv != c)
            for (int j = 0; j < 6; ++j) {
                Cx t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t;
                t = inv[c][j]; inv[c][j] = inv[piv][j]; inv[piv][j] = t;
            }
        const Cx p = a[c][c];
        const double den = p.r * p.r + p.i * p.i;
        const Cx pinv = {p.r / den, -p.i / den};
        for (int j = 0; j < 6; ++j) {
            a[c][j] = cmul(a[c][j], pinv);
            inv[c][j] = cmul(inv[c][j], pinv);
        }
        for (int r = 0; r < 6; ++r) {
            if (r == c) continue;
            const Cx f = a[r][c];
            for (int j = 0; j < 6; ++j) {
                const Cx t1 = cmul(f, a[c][j]), t2 = cmul(f, inv[c][j]);
                a[r][j].r -= t1.r; a[r][j].i -= t1.i;
                inv[r][j].r -= t2.r; inv[r][j].i -= t2.i;
            }
        }
    }
    return ok;
}

template <class S>
__global__ __launch_bounds__(CLOVER_WG) void sap_clover_kernel(Geom geo, const double *tclov, double kappa, S *out,
                                                               float *scale, int *singular) {
    const int64_t t = (int64_t)blockIdx.x * CLOVER_WG + threadIdx.x;
    if (t >= geo.V) return;
    const int64_t bp = t / geo.Vbh;
    const int s = (int)(t - bp * geo.Vbh);
    double tp[72], packed[72];
    load_site<double, 72>(tclov, nullptr, bp, s, geo.Vbh, tp);
    if ((bp & 1) == 0) {
        for (int k = 0; k < 72; ++k) packed[k] = kappa * tp[k];
    } else {
        for (int k = 0; k < 2; ++k) {
            Cx a[6][6], inv[6][6];
            unpack6(tp + 36 * k, a);
            for (int i = 0; i < 6; ++i)
                for (int j = 0; j < 6; ++j) {
                    a[i][j].r *= kappa;
                    a[i][j].i *= kappa;
                }
            for (int i = 0; i < 6; ++i) a[i][i].r += 1.0;
            if (!invert6(a, inv)) *singular = 1;
            for (int i = 0; i < 6; ++i) inv[i][i].r -= 1.0;
            // Hermitian by construction; average the two triangles against rounding
            for (int i = 0; i < 6; ++i)
                for (int j = i + 1; j < 6; ++j) {
                    inv[i][j].r = 0.5 * (inv[i][j].r + inv[j][i].r);
                    inv[i][j].i = 0.5 * (inv[i][j].i - inv[j][i].i);
                }
            pack6(inv, packed + 36 * k);
        }
    }
    store_site<double, 72>(out, scale, bp, s, geo.Vbh, packed);
}

static dim3 cgrid(const Geom &geo) { return dim3((unsigned)((geo.V + CLOVER_WG - 1) / CLOVER_WG)); }

hipError_t launch_clover_build(const Geom &geo, const double *links, double csw, double *tclov, hipStream_t st) {
    if (geo.V == 0) return hipSuccess;
    hipLaunchKernelGGL(clover_build_kernel, cgrid(geo), dim3(CLOVER_WG), 0, st, geo, links, csw, tclov);
    return hipGetLastError();
}

hipError_t launch_clover_pack(const Geom &geo, const double *canon, double *tclov, hipStream_t st) {
    if (geo.V == 0) return hipSuccess;
    hipLaunchKernelGGL(clover_pack_kernel, cgrid(geo), dim3(CLOVER_WG), 0, st, geo, canon, tclov);
    return hipGetLastError();
}

hipError_t launch_sap_clover(const Geom &geo, const double *tclov, double kappa, Fld out, int *singular,
                             hipStream_t st) {
    if (geo.V == 0) return hipSuccess;
    if (out.prec == P64)
        hipLaunchKernelGGL((sap_clover_kernel<double>), cgrid(geo), dim3(CLOVER_WG), 0, st, geo, tclov, kappa,
                           (double *)out.data, nullptr, singular);
    else if (out.prec == P32)
        hipLaunchKernelGGL((sap_clover_kernel<float>), cgrid(geo), dim3(CLOVER_WG), 0, st, geo, tclov, kappa,
                           (float *)out.data, nullptr, singular);
    else
        hipLaunchKernelGGL((sap_clover_kernel<half_t>), cgrid(geo), dim3(CLOVER_WG), 0, st, geo, tclov, kappa,
                           (half_t *)out.data, out.scale, singular);
    return hipGetLastError();
}

}  // namespace sapdd
