// kernels.hpp - host-side launchers of the sapdd device kernels (one declaration per
// kernel family). All launchers enqueue on `stream` and return the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "core.hpp"

namespace sapdd {

enum Prec { P64 = 0, P32 = 1, P16 = 2 };

// Untyped view of a block-tiled field: data in `prec` plus per-site scales (FP16 only).
struct Fld {
    void *data;
    float *scale;
    int prec;
};

// ---- layout (layout.hip)
// Canonical FP64 array (ncomp = 24 spinor, 72 links) -> block-tiled field, nfield copies
// (per-field strides V * ncomp / V).
hipError_t launch_pack(const Geom &geo, int ncomp, int nfield, const double *canon, Fld out, hipStream_t st);
hipError_t launch_unpack(const Geom &geo, int ncomp, int nfield, Fld in, double *canon, hipStream_t st);
// Block-tiled FP64 field -> another storage precision (same layout).
hipError_t launch_convert(const Geom &geo, int ncomp, int nfield, const double *in, Fld out, hipStream_t st);
// dst[i] = src[i] for n bytes (16-byte vector copies plus a tail).
hipError_t launch_copy(const void *src, void *dst, int64_t n, hipStream_t st);

// ---- clover (clover.hip)
// T(x) from the block-tiled FP64 links (periodic closure of every plaquette).
hipError_t launch_clover_build(const Geom &geo, const double *links, double csw, double *tclov, hipStream_t st);
// T(x) from the canonical 12x12 complex form.
hipError_t launch_clover_pack(const Geom &geo, const double *canon, double *tclov, hipStream_t st);
// X for the SAP kernels: kappa T on even sites, (1 + kappa T)^-1 - 1 on odd sites,
// written in out.prec. Sets *singular (device int) to 1 if a pivot falls below 1e-12.
hipError_t launch_sap_clover(const Geom &geo, const double *tclov, double kappa, Fld out, int *singular,
                             hipStream_t st);

// ---- operators (dslash.hip)
struct DslashIO {
    Fld in;            // spinor of rhs r at in + r * in_stride * V * 24 (scales: * V)
    Fld out;           // idem with out_stride
    const double *sub; // if set (FP64 out only): out = sub - M in, rhs stride sub_stride
    double *part;      // if set: per-workgroup partial |out|^2, [nact][dslash_full_partials]
    const int *active; // if set: rhs index of each of the nact slots
    int nact;
    int in_stride, out_stride, sub_stride;  // in units of one spinor field
    const double *kappa;                    // if set: per-rhs kappa (device), else the scalar
};
// Number of partial sums launch_dslash_full writes per RHS slot.
int dslash_full_partials(const Geom &geo);
// out = M in over the whole lattice. links/clov in `lprec` (FP64: links + T in FP64).
hipError_t launch_dslash_full(const Geom &geo, Fld links, Fld tclov, double kappa, const DslashIO &io,
                              hipStream_t st);
// out = M_B in (hops between blocks dropped), one workgroup per (block, rhs).
hipError_t launch_dslash_block(const Geom &geo, Fld links, Fld tclov, double kappa, Fld in, Fld out, int nrhs,
                               hipStream_t st);

// ---- block operator with two-row links (links12.hip)
// Rows 0 and 1 of every link of the FP64 block-tiled field (48 reals per site) in out.prec
// (P32 or P16 with per-site scales).
hipError_t launch_links12_pack(const Geom &geo, const double *links64, Fld out, hipStream_t st);
// out = M_B in with the links in that form (third rows rebuilt in the kernel), FP32 or
// FP16 storage throughout.
hipError_t launch_dslash_block12(const Geom &geo, Fld links12, Fld tclov, double kappa, Fld in, Fld out, int nrhs,
                                 hipStream_t st);

// ---- Schwarz sweep (sap.hip)
struct SapArgsHost {
    Fld links;                // storage-precision links
    const void *const *X;     // per-rhs clover X (device array of nrhs pointers)
    const float *const *Xsc;  // per-rhs clover scales (FP16) or null
    const double *kappa;      // per-rhs kappa (device)
    const double *eta;        // FP64 block-tiled input, stride V * 24 per rhs
    const double *eta_scale;  // factor applied to eta of rhs r: eta_scale[r * eta_scale_stride], or null
    int eta_scale_stride;
    int eta_stride_rhs;       // in units of V * 24 doubles
    Fld rres;                 // even-site residual, stride V * 12 per rhs (scales V / 2)
    Fld delta;                // last correction, stride V * 24 per rhs
    void *psi;                // output, P32 or P64 per psi_prec, stride V * 24 per rhs
    int psi_prec;
    int psi_stride_rhs;       // in units of V * 24
    const int *active;        // slot -> rhs
    int nact;
    int nmr;
};
// One half-sweep over the blocks of `colour`. mode 0: rho = eta; mode 1: rho = eta +
// gather; mode 2: rho = stored residual + gather. write_state = 0 skips storing the
// residual and correction (last half-sweep).
hipError_t launch_sap_half(const Geom &geo, const SapArgsHost &a, int colour, int mode, int write_state,
                           hipStream_t st);

// ---- FP64 Krylov kernels (blas.hip)
// Vectors are complex FP64 in the block-tiled layout, n = 12 V complex entries each
// (a flat complex array: the layout keeps real and imaginary parts adjacent). For the
// rhs of slot q: basis vector i at vbase + rhs * rstride + i * vstride (doubles), stored
// unnormalised with the factor vscale[rhs * vsstride + i]; w at w + rhs * wstride.
struct CgsArgs {
    const double *vbase;
    int64_t vstride, rstride;
    const double *vscale;
    int vsstride;
    double *w;
    int64_t wstride;
    const double *coef;  // complex coefficients of rhs r at coef + r * cstride (modes 1, 2)
    int cstride;
    double *part;        // partial sums [nact][blas_partials][nval]
    const int *active;
    int nact;
    int v0, nv;          // basis vectors v0 .. v0 + nv - 1 (nv <= 16)
    int64_t n;
    double skip_tol;     // mode 2: skip the pass where |c|^2 <= skip_tol |w|^2 (see launch_cgs)
};
// Workgroups per rhs slot used by the Gram-Schmidt passes.
int blas_partials(int64_t n, int nact);
// mode 0: partial <v_i, w>; mode 1: w -= sum_i coef_i s_i v_i, then partials <v_i, w>
// and, as value 2 nv, |w|^2; mode 2: w -= sum_i coef_i s_i v_i, then partial |w|^2.
// Coefficient i of the pass is coef[2 (v0 + i)] (re, im). Mode 2 with skip_tol > 0 and
// nv > 0 reads |w|^2 at coef[2 (v0 + nv)] (mode 1's last value): where the correction is
// negligible, sum |coef_i|^2 <= skip_tol |w|^2, a slot's pass leaves w as it is and its
// partials sum to that |w|^2 exactly.
hipError_t launch_cgs(int mode, const CgsArgs &a, hipStream_t st);
// For every slot: v_k = sum over wg of part[slot][k][wg] (fixed order), times
// mul[rhs * mstride + v0 + k / 2] if mul is set (for an odd nval not the last value,
// which is a norm); written to out[rhs * ostride + k].
// If isq is set, isq[rhs * istride] = 1 / sqrt(v_0) (0 if v_0 <= 0).
hipError_t launch_reduce(const double *part, int nwg, int nval, const int *active, int nact, double *out,
                         int ostride, const double *mul, int mstride, int v0, double *isq, int istride,
                         hipStream_t st);
// In place v_l <- sum_{i < nin} s_i v_i P_il (l < nout <= nin) for the FP64 vectors of
// every listed slot (n complex entries; slot rhs at base + rhs * rstride, vector i at
// + i * vstride doubles); s_i = vscale[rhs * vsstride + i] (1 if vscale is null), which
// is then set to 1 for i < nout. P: column-major, leading dimension ld, complex, at
// P + rhs * pstride doubles. nin <= 17.
hipError_t launch_recombine(double *base, int64_t rstride, int64_t vstride, const double *vscale, int vsstride,
                            const double *P, int64_t pstride, int ld, int nin, int nout, const int *active, int nact,
                            int64_t n, hipStream_t st);
// x[rhs] += sum_j y[rhs][j] z_j[rhs]: y complex at y + rhs * ystride, z in P32 or P64 at
// z + (rhs * zstride_rhs + j * zstride_j) elements.
hipError_t launch_zupdate(double *x, int64_t xstride, const void *z, int zprec, int64_t zstride_j,
                          int64_t zstride_rhs, const double *y, int ystride, int nz, const int *active, int nact,
                          int64_t n, int vbh, hipStream_t st);

// ---- two-level multigrid (mg.hip)
constexpr int MG_NVEC_MAX = 16;  // test vectors (coarse dofs per aggregate and chirality)
constexpr int MG_IMAX = 24;      // coarse GMRES steps
constexpr int MG_CWG = 256;      // workgroup of the coarse kernels
// Colouring of the block grid for probing the coarse operator: colour of block
// coordinates g = sum_mu (g_mu mod m_mu) * prod_{nu < mu} m_nu, n colours.
struct MgColouring {
    int m[4];
    int n;
};
int mg_colour_of(const int g[4], const MgColouring &cl);
// In place: per aggregate and chirality, Gram-Schmidt (twice) over nvec FP64 fields.
hipError_t launch_mg_orth(const Geom &geo, double *w, int nvec, hipStream_t st);
// out(rhs) = P^H in(rhs): FP64 fields (stride in doubles) -> FP32 complex coarse vectors
// (stride in complex numbers); rhs = active[slot] (slot if active is null).
hipError_t launch_mg_restrict(const Geom &geo, int nvec, const double *in, int64_t in_stride, const float *P,
                              float2 *out, int64_t out_stride, const int *active, int nact, hipStream_t st);
// out(rhs) = P sum_{i < nb} coef(rhs)[i] basis(rhs)[i] (coef null: P basis(rhs)), FP64
// output (stride in doubles).
hipError_t launch_mg_prolong_basis(const Geom &geo, int nvec, const float *P, const float2 *basis, int64_t bstride,
                                   int64_t vstride, const double *coef, int64_t cstride, int nb, double *out,
                                   int64_t out_stride, const int *active, int nact, hipStream_t st);
// out(col) = P e for e = 1 in coarse column k0 + col on the aggregates of colour q
// (col < ncol; out stride V * 24 doubles).
hipError_t launch_mg_prolong_probe(const Geom &geo, int nvec, const float *P, int q, const MgColouring &cl, int k0,
                                   int ncol, double *out, hipStream_t st);
// D_c columns k0 .. k0 + ncol - 1 from the restricted probe results R[col][b][row].
hipError_t launch_mg_scatter(const Geom &geo, const float2 *R, int ncol, int k0, int K, int q,
                             const MgColouring &cl, float2 *Dc, hipStream_t st);
// y(rhs) += alpha * scale[rhs * sstride] * x(rhs) (scale may be null): y FP64 or FP32,
// x FP64, strides in elements of each.
hipError_t launch_mg_axpy(const Geom &geo, Fld y, int64_t ystride, const double *x, int64_t xstride, double alpha,
                          const double *scale, int sstride, const int *active, int nact, hipStream_t st);
// Coarse GMRES state of the listed systems (all buffers per rhs, indexed by rhs).
struct MgGmres {
    const float2 *Dc;  // coarse operator
    int K;             // 2 nvec
    int grid[4];       // block grid
    int64_t Nd;        // aggregates
    int nwa, nwc;      // workgroups per system of the operator and Gram-Schmidt kernels
    int pstride;       // partials stride per value (>= nwa, nwc)
    float2 *basis;     // basis(rhs)[i] at basis + rhs * bstride + i * vstride, i <= MG_IMAX, then
                       // the two slots of the unscaled operator products

    int64_t bstride, vstride;
    float2 *rc;        // right-hand side(rhs) at rc + rhs * vstride
    float2 *xc;        // solution(rhs) at xc + rhs * vstride
    double *pn;        // [rhs][MG_IMAX + 1][pstride] |v_i|^2 partials
    double *pd;        // [rhs][2][2 MG_IMAX][pstride] Gram-Schmidt partials
    double *H;         // [rhs][MG_IMAX][MG_IMAX + 1] complex, column-major Hessenberg
    double *sc;        // [rhs][MG_IMAX + 1] 1 / |v_i|
    double *beta;      // [rhs] |rhs|
    double *coef;      // [rhs][MG_IMAX] complex: a cycle's correction = sum_i coef[i] basis[i]
    int fused;         // 1: one launch per Arnoldi step, 0: two
    const int *active;
};
void mg_coarse_tiling(const Geom &geo, int K, int *nwa, int *nwc);
constexpr int MG_BASIS_SLOTS = MG_IMAX + 3;     // coarse vectors per system: basis and products
// cycles cycles of restarted GMRES(k) from zero on D_c xc = rc for every listed system.
hipError_t launch_mg_coarse_gmres(const MgGmres &G, int nact, int k, int cycles, hipStream_t st);
// rc(rhs) = in(rhs) rounded to FP32, in complex FP64 at in + rhs * istride.
hipError_t launch_mg_load(const MgGmres &G, int nact, const double *in, int64_t istride, hipStream_t st);
// out(rhs) = xc(rhs) as complex FP64 at out + rhs * ostride.
hipError_t launch_mg_solution(const MgGmres &G, int nact, double *out, int64_t ostride, hipStream_t st);

}  // namespace sapdd
