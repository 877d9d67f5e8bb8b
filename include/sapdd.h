/*
 * sapdd.h - C ABI of the MI355X (gfx950) Schwarz-preconditioned Wilson-clover solver.
 *
 * The library implements the domain-decomposition solver summarised in arxiv 1502.04025,
 * Sec. 3.1: the Wilson-clover Dirac operator M, the multiplicative Schwarz (Schwarz
 * alternating procedure, SAP) preconditioner over red/black coloured blocks with each
 * block solved approximately by minimal-residual (MR) iterations on its even-odd reduced
 * operator, and an outer flexible GMRES (FGMRES) in double precision. The data-layout
 * (structure of arrays, Sec. 3.2) and half-precision storage (Sec. 3.3) choices of the
 * paper are re-made for the GPU: a block-tiled even-odd SoA layout in HBM and optional
 * FP16 storage with one FP32 scale per site.
 *
 * Conventions shared by every call
 * ---------------------------------
 * Lattice dims[4] = {Lx, Ly, Lz, Lt}; sites are ordered x fastest, then y, z, t.
 * Boundary conditions: periodic in x, y, z; antiperiodic in t when antiperiodic_t != 0.
 * Dirac basis: DeGrand-Rossi (chiral, gamma_5 = diag(1, 1, -1, -1)).
 * Operator (kappa normalisation):
 *   (M psi)(x) = (1 + kappa T(x)) psi(x)
 *       - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * with the sign -1 on hops across the time boundary (antiperiodic t) and the clover term
 * T(x) = -c_sw sum_{mu<nu} gamma_mu gamma_nu (x) F_mu,nu(x), F = (Q - Q^+)/8 made traceless,
 * Q the sum of the four plaquettes in the (mu, nu) plane based at x.
 *
 * Canonical host/device arrays (all IEEE double, complex numbers interleaved re, im):
 *   links   [t][z][y][x][mu][3][3] complex   (mu = 0..3 for x, y, z, t; U[a][b], row a)
 *   spinor  [rhs][t][z][y][x][4][3] complex  (spin, colour)
 *   clover  [t][z][y][x][12][12] complex     (T(x), row/column index 3*spin + colour)
 *
 * Pointers are host memory unless SAPDD_DEVICE_PTRS is set in `flags`, in which case they
 * are device memory of the context's device (for instance torch tensor data pointers).
 * Caller buffers stay owned by the caller. Fields are copied into library-owned device
 * memory on load and released by sapdd_free_field. Every call is synchronous with respect
 * to the context's stream: it enqueues its work on that stream and waits for it before
 * returning.
 *
 * Errors: every int-returning call returns SAPDD_OK (0) or a negative status; the message
 * of the last failure on a context is available from sapdd_last_error. Nothing throws or
 * aborts across the ABI. One context must not be used from two host threads at once.
 */
#ifndef SAPDD_H
#define SAPDD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sapdd_ctx sapdd_ctx;     /* device, stream, workspaces, last error      */
typedef struct sapdd_field sapdd_field; /* one resident gauge field and its clover term */
typedef struct sapdd_batch sapdd_batch; /* continuous-batching solver state (slots)    */
typedef struct sapdd_mg sapdd_mg;       /* two-level multigrid preconditioner          */

enum {
    SAPDD_OK = 0,
    SAPDD_EINVAL = -1,    /* bad argument or unsupported shape                      */
    SAPDD_ENOMEM = -2,    /* device allocation failed                               */
    SAPDD_EDEVICE = -3,   /* HIP runtime error                                      */
    SAPDD_ENOCONV = -4,   /* solver hit max_iter; x and stats hold the best iterate */
    SAPDD_ESINGULAR = -5, /* a clover block 1 + kappa T is singular (pivot < 1e-12) */
    SAPDD_ENAN = -6,      /* NaN or Inf in a residual                               */
    SAPDD_EFULL = -7      /* no free slot in a batch                                */
};

/* Storage precisions. SAPDD_F16 stores every site with one FP32 scale (max |value| of the
 * site). sap_prec additionally takes SAPDD_F16_LINKS: links and clover in FP16 (with the
 * site scale), the Schwarz residual and corrections in FP32 - the half-precision mode of
 * Sec. 3.3, which keeps the spinors in single precision. */
enum { SAPDD_F64 = 0, SAPDD_F32 = 1, SAPDD_F16 = 2, SAPDD_F16_LINKS = 3 };

enum {
    SAPDD_DEVICE_PTRS = 1, /* array arguments are device pointers              */
    SAPDD_USE_X0 = 2,      /* sapdd_solve starts from the x passed in, not 0    */
    SAPDD_NO_GRAPH = 4,    /* sapdd_solve launches the SAP sweep without a graph */
    SAPDD_LINKS12 = 8,     /* sapdd_apply_block_D: links stored as their first two
                            * rows, the third rebuilt in the kernel (FP32/FP16)  */
    SAPDD_ELASTIC = 16     /* sapdd_batch_create: a slot's device memory is committed
                            * when the slot is first admitted, kept when it is taken
                            * (the next add reuses it) and given back by
                            * sapdd_batch_trim; uncommitted slots cost address
                            * space only. The physical memory comes in chunks of at
                            * most 64 MiB from a pool the elastic batches of the
                            * process share per device; trimmed chunks return to it
                            * and serve any elastic batch's next commit, and the pool
                            * frees them when the device's last elastic batch is
                            * destroyed. An elastic batch also allocates at creation
                            * the field's 16 clover-inverse buffers for its
                            * precision, so admitting a new kappa allocates nothing */
};

/* Solver parameters (Sec. 3.1 names the pieces; Sec. 3.7 uses 4-5 MR iterations and
 * 16 Schwarz cycles). block[] must equal the blocking the field was loaded with or be
 * all zero (use the field's). */
typedef struct {
    int block[4];   /* Schwarz block extents Bx, By, Bz, Bt                         */
    int nmr;        /* MR iterations per block solve (>= 1)                        */
    int ncy;        /* SAP cycles, each = colour 0 then colour 1 (>= 1)            */
    int restart;    /* FGMRES restart length m (1..16)                             */
    int max_iter;   /* cap on outer iterations (preconditioner applications)       */
    double tol;     /* target true relative residual |b - M x| / |b|               */
    int sap_prec;   /* storage inside SAP: SAPDD_F64, SAPDD_F32, SAPDD_F16 (links,
                     * clover and spinors) or SAPDD_F16_LINKS (FP16 links and clover,
                     * FP32 spinors)                                                   */
    int flags;      /* SAPDD_DEVICE_PTRS | SAPDD_USE_X0 | SAPDD_NO_GRAPH          */
    int deflate;    /* deflated restarts (Sec. 3.1, flexible GMRES with deflated
                     * restarts): k harmonic Ritz vectors of the cycle's Hessenberg
                     * matrix, those of smallest modulus, are kept across each full
                     * restart (0 = plain restarts; 0 <= k < restart). With k > 0 the
                     * preconditioned vectors Z are held in FP64 whatever sap_prec is.  */
    double gap;     /* reliable-update gap (0 = 10): at the end of every restart cycle
                     * the FP64 true residual |b - M x| is compared with the cycle's
                     * implicit one (the least-squares residual the Arnoldi relation
                     * carries); when true > gap * implicit the implicit residual is not
                     * trusted and the next cycle restarts plainly from the true
                     * residual, dropping a deflated basis (counted in
                     * sapdd_stats.gap_restarts).                                       */
} sapdd_params;

/* Per right-hand-side result of sapdd_solve. Times are seconds of device time
 * (HIP events) spent in each phase, summed over the solve; a batched solve attributes
 * the whole batch's phase time to every RHS in it. */
typedef struct {
    int iters;              /* outer iterations (preconditioner applications)        */
    int restarts;           /* completed restart cycles                              */
    int converged;          /* 1 if true_relres <= tol                               */
    double true_relres;     /* |b - M x| / |b| recomputed in FP64 at the end         */
    double implicit_relres; /* least-squares residual estimate at the last step      */
    double t_total;         /* wall time of the call                                 */
    double t_sap, t_dslash, t_gs, t_host;
    int gap_restarts;       /* cycles whose true residual exceeded gap x implicit    */
} sapdd_stats;

/* Create a context on HIP device `device`, enqueueing on `hip_stream` (a hipStream_t;
 * NULL = the device's null stream). */
int sapdd_create(int device, void *hip_stream, sapdd_ctx **out);
void sapdd_destroy(sapdd_ctx *ctx);
/* Message of the last failed call on ctx ("" if none). Valid until the next call. */
const char *sapdd_last_error(const sapdd_ctx *ctx);

/* Sec. 3.2 (data layout) and Sec. 3.5 (two-coloured domains): upload a gauge field
 * (canonical links, host or device per flags, copied into library-owned memory freed by
 * sapdd_free_field) and fix its device layout: the lattice is tiled
 * by Schwarz blocks of extents block[] (each even and >= 2, dividing dims, with an even
 * number of blocks per direction so the blocks two-colour the lattice, Sec. 3.5 footnote).
 * Supported block shapes: 2x2x2x2, 4x4x4x4, 8x4x4x4. The clover term starts at zero.
 * The library caches the SAP clover inverse of up to 16 kappas on the field and reuses
 * an evicted one's memory for the next kappa in stream order, so calls that use one
 * field must not overlap on different streams. */
int sapdd_load_gauge(sapdd_ctx *ctx, const int dims[4], const int block[4], const double *links,
                     int antiperiodic_t, int flags, sapdd_field **out);
/* Sec. 3.1 (the operator is Wilson-clover): build the clover term T(x) on the device from
 * the resident links, with coefficient c_sw >= 0, in the form stated at the top of this
 * header (four same-orientation plaquette leaves per plane, traceless F). Replaces any
 * clover loaded before and drops the field's derived low-precision and per-kappa copies.
 * EINVAL for c_sw < 0 or a null argument; EDEVICE on a HIP error. */
int sapdd_compute_clover(sapdd_ctx *ctx, sapdd_field *field, double csw);
/* Sec. 3.1 (Wilson-clover operator): upload a caller-made T(x) (canonical clover layout,
 * FP64 host or device array per flags, copied; the caller keeps ownership). Only the two
 * chiral 6x6 blocks (spins 0-1 and 2-3) are read; the entries coupling them must be zero
 * in the Dirac basis above. EINVAL for a null argument; EDEVICE on a HIP error. */
int sapdd_load_clover(sapdd_ctx *ctx, sapdd_field *field, const double *clover, int flags);
/* Free a field. The context's kept sapdd_solve batch on it goes with it; batches and
 * multigrid objects the caller made on the field must be destroyed first. */
int sapdd_free_field(sapdd_ctx *ctx, sapdd_field *field);

/* Sec. 3.1 (the Wilson-clover operator M the solver inverts; Sec. 3.7 counts it at 1848
 * flop per site): out = M in for nrhs canonical spinors ([nrhs][t][z][y][x][4][3]
 * complex128, host or device per flags), with links, clover and spinors held in storage
 * precision `prec` (arithmetic in FP64 for SAPDD_F64, FP32 otherwise; SAPDD_F16 stores
 * every site with one FP32 scale, the half-precision storage of Sec. 3.3). in and out
 * may not overlap; the caller owns both. EINVAL for nrhs < 1, a bad precision or a null
 * argument; ENOMEM if a workspace cannot be allocated. */
int sapdd_apply_D(sapdd_ctx *ctx, const sapdd_field *field, double kappa, int prec, int nrhs,
                  const double *in, double *out, int flags);
/* Sec. 3.1 (the splitting of M into its block-diagonal part and the remainder): out =
 * M_B in, M with every hop between two different Schwarz blocks removed; same arguments,
 * layouts, ownership and errors as sapdd_apply_D.
 * With SAPDD_LINKS12 in flags (FP32 or FP16 only) every link is read as its first two
 * rows and the third is rebuilt as the complex conjugate of their cross product: a third
 * fewer link bytes, exact for special unitary links (the library does not check that).
 * The two-row copy is made on first use and kept with the field. */
int sapdd_apply_block_D(sapdd_ctx *ctx, const sapdd_field *field, double kappa, int prec,
                        int nrhs, const double *in, double *out, int flags);
/* Sec. 3.1 (the multiplicative Schwarz preconditioner: red/black domains, each solved
 * approximately by MR with even-odd preconditioning) and Sec. 3.3 (half-precision
 * storage): out = SAP(in), params->ncy cycles of params->nmr MR steps per block solve over
 * colour 0 then colour 1, starting from zero; kappa[nrhs] may differ per right-hand side
 * (all of them share every launch). in and out: nrhs canonical spinors (FP64,
 * host or device per params->flags, caller-owned, not overlapping); storage inside the
 * sweep params->sap_prec (SAPDD_F16: one FP32 scale per site), arithmetic FP32 below FP64.
 * EINVAL for bad params (block differs from the field's, nmr or ncy < 1) or kappa <= 0; ESINGULAR if
 * 1 + kappa T is singular on some site; ENOMEM if a workspace cannot be allocated. */
int sapdd_sap(sapdd_ctx *ctx, const sapdd_field *field, const double *kappa, const sapdd_params *params,
              int nrhs, const double *in, double *out);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sapdd_sap with every workspace (the
 * packed input and output, the Schwarz residual and correction, the clover inverse per
 * distinct kappa, low-precision links when the field has none yet, per-rhs metadata) in
 * a fixed 256 MiB array of device memory that each GPU holds from the library's first use
 * until the process ends. The call allocates nothing, on the device or the host, and
 * otherwise behaves as sapdd_sap with the same arguments (bit-identical output). Limits:
 * in and out must be device pointers (SAPDD_DEVICE_PTRS in params->flags), nrhs <= 16,
 * and the workspaces must fit in 256 MiB (for example 16^3 x 32 with one right-hand side
 * in any precision); beyond them it returns SAPDD_EINVAL with the size it would need.
 * All calls on one GPU share the array: calls that overlap in time on one GPU (two
 * contexts, two host threads or two streams) race and must be serialised by the caller.
 * SAPDD_EDEVICE if the array has no device address on this device. */
int sapdd_sap_noalloc(sapdd_ctx *ctx, const sapdd_field *field, const double *kappa,
                      const sapdd_params *params, int nrhs, const double *in, double *out);
/* Sec. 3.1 (the outer flexible GMRES, preconditioned by the Schwarz procedure, in FP64
 * with lower-precision preconditioning, Sec. 3.3): solve M x = b for nrhs right-hand
 * sides with SAP-preconditioned FGMRES(m) (a batch of nrhs slots stepped to completion;
 * the context keeps it for later calls). b and x: canonical spinors, host or device per
 * params->flags, caller-owned; every RHS finishes on its FP64 true residual.
 * kappa[nrhs] may differ per RHS. x holds nrhs canonical spinors (read as the start
 * vector if SAPDD_USE_X0). stats may be NULL, else it has nrhs entries. Returns
 * SAPDD_ENOCONV if some RHS missed tol within max_iter. */
int sapdd_solve(sapdd_ctx *ctx, const sapdd_field *field, const double *kappa,
                const sapdd_params *params, int nrhs, const double *b, double *x,
                sapdd_stats *stats);

/* Continuous batching (the serving form of the solver). A batch holds up to `capacity`
 * right-hand sides on one field, each with its own kappa and its own FP64 FGMRES(m)
 * state. sapdd_batch_step runs one restart cycle for every unfinished slot: one SAP
 * launch sequence (replayed from a HIP graph captured per slot count and Arnoldi step,
 * unless SAPDD_NO_GRAPH), one operator launch and the Gram-Schmidt passes per Arnoldi
 * step serve the whole batch (classical Gram-Schmidt twice; a slot skips the second
 * correction where its coefficients are below 1e-9 of the corrected vector's norm, and
 * its Hessenberg column then takes the first pass alone), and a true FP64 residual at
 * the end of the cycle decides convergence. Right-hand sides join with sapdd_batch_add and leave with
 * sapdd_batch_take between steps. A slot's result does not depend on which other slots
 * share the batch (slots are processed independently, reductions in a fixed order).
 * The batch allocates its device memory at creation (sapdd_solve_footprint bytes for
 * `capacity` RHS, clover inverses per kappa excluded; with SAPDD_ELASTIC the slots'
 * memory only as slots are admitted) and uses the context's stream; a batch and its
 * context belong to one host thread at a time. */
int sapdd_batch_create(sapdd_ctx *ctx, const sapdd_field *field, const sapdd_params *params, int capacity,
                       sapdd_batch **out);
int sapdd_batch_destroy(sapdd_batch *batch);
/* Device memory the batch holds now (bytes): its fixed workspaces, plus, with
 * SAPDD_ELASTIC, the memory committed for its slots (in use, or kept after a take until
 * sapdd_batch_trim). *slot_bytes (if not NULL)
 * receives the most one more admitted slot can commit (0 for a batch allocated whole at
 * creation). Admission by footprint across batches (the serving loop) reads these; the
 * clover inverse of a new kappa (sapdd_solve_footprint counts it) comes on top. -1 for
 * a NULL batch. */
long long sapdd_batch_memory(const sapdd_batch *batch, long long *slot_bytes);
/* SAPDD_ELASTIC: give back the device memory of free slots that still hold it from an
 * earlier use, keeping at most `keep` of them committed (keep = 0 releases all). The
 * chunks go to the elastic batches' shared pool (above), not to the device: another
 * elastic batch then commits them without allocating. Waits for the batch's stream
 * first. Returns the bytes released (0 for a batch allocated whole), -1 for a NULL
 * batch or keep < 0, a negative error code if the stream failed. */
long long sapdd_batch_trim(sapdd_batch *batch, int keep);
/* Admit one right-hand side b (canonical spinor; x0 = start vector or NULL for zero;
 * flags: SAPDD_DEVICE_PTRS). An elastic batch takes a free slot that still holds its
 * memory first and commits a new one only if there is none. The call waits for the
 * device only to check the clover term of a kappa new to the field (singular pivot) and,
 * with host arrays, for their copy; device arrays are read on the context's stream after
 * it returns. |b| is read back by the next sapdd_batch_step (for every slot added since,
 * at once): a zero b finishes there with x = 0, a non-finite one with SAPDD_ENAN at
 * take. Returns SAPDD_EFULL if every slot is taken, SAPDD_ENOMEM if an elastic batch
 * cannot commit the slot's memory (nothing stays committed). */
int sapdd_batch_add(sapdd_batch *batch, double kappa, const double *b, const double *x0, int flags, int *slot);
/* One restart cycle for every unfinished slot; *running = slots still unfinished. */
int sapdd_batch_step(sapdd_batch *batch, int *running);
/* 1 if the slot is finished (converged, failed or out of iterations), 0 if running;
 * fills stats when not NULL. */
int sapdd_batch_poll(const sapdd_batch *batch, int slot, sapdd_stats *stats);
/* Copy the slot's solution to x (canonical; flags: SAPDD_DEVICE_PTRS), fill stats and
 * free the slot. Taking an unfinished slot cancels it: x is then the iterate of its last
 * completed restart cycle, a resume point to pass back later as x0 (SAPDD_USE_X0). */
int sapdd_batch_take(sapdd_batch *batch, int slot, double *x, int flags, sapdd_stats *stats);

/* Two-level multigrid with the Schwarz procedure as smoother (Sec. 2.6: the group's
 * multigrid solver is a Krylov method preconditioned by a multigrid cycle whose smoother
 * is the domain-decomposition preconditioner of Sec. 3.1; the rest follows the adaptive
 * aggregation method the paper cites).
 *   Aggregates: the field's Schwarz blocks, each split into its two chiralities (spins
 *     0-1 and 2-3, gamma_5 = +1 and -1).
 *   Test vectors: nvec fields given by the caller (random numbers are inputs, not drawn
 *     here), each smoothed setup_iters times by v <- v - SAP(M v).
 *   Interpolation P: on every aggregate and chirality the test vectors orthonormalised
 *     by Gram-Schmidt in index order; coarse index k = s * nvec + j (chirality s, vector
 *     j), K = 2 nvec coarse dofs per aggregate. Stored in FP32.
 *   Coarse operator: D_c = P^H M P (Galerkin), nine K x K blocks per aggregate (itself
 *     and its forward and backward neighbour in each direction), FP32, built on the
 *     device by applying the FP64 operator to interpolated unit vectors.
 *   Preconditioner B(r) = e + SAP(r - M e), e = P GMRES(D_c, P^H r): coarse_cycles
 *     cycles of restarted GMRES(coarse_iters) from zero, run on the device, then one SAP
 *     application (smoother params: nmr, ncy, sap_prec) on the remaining residual.
 * Coarse vectors in the canonical form are complex [aggregate][K], aggregates in block
 * order (x fastest), as complex128. A multigrid object belongs to its field and kappa
 * and must be destroyed before the field is freed. */
typedef struct {
    int nvec;         /* test vectors per aggregate and chirality: even, 2..16          */
    int setup_iters;  /* smoothing passes per test vector before P is built (>= 0)     */
    int coarse_iters; /* GMRES steps per coarse restart cycle (1..24)                  */
    int coarse_cycles;/* restart cycles of every coarse solve (0..64; 0 = 1)           */
    int coarse_form;  /* 0: two kernel launches per coarse Arnoldi step (for batches of  */
                      /* systems), 1: one launch per step, each workgroup correcting the  */
                      /* rows it applies the stencil to (for a single system). Both run   */
                      /* classical Gram-Schmidt; results agree to rounding. Fixed per     */
                      /* object, so a system gets the same bits alone and in any batch.   */
} sapdd_mg_params;
/* Build P and D_c for (field, kappa). vecs: nvec canonical spinors (flags:
 * SAPDD_DEVICE_PTRS). smoother supplies nmr, ncy and sap_prec of the smoothing passes
 * and of sapdd_mg_precond. Blocks must have at most 512 sites. */
int sapdd_mg_setup(sapdd_ctx *ctx, sapdd_field *field, double kappa, const sapdd_params *smoother,
                   const sapdd_mg_params *mgp, const double *vecs, int flags, sapdd_mg **out);
int sapdd_mg_destroy(sapdd_mg *mg);
/* The nvec interpolation fields (FP32 values widened to FP64) as canonical spinors:
 * column s * nvec + j of P is the chirality-s half of field j on every aggregate. */
int sapdd_mg_prolongator(sapdd_mg *mg, double *fields, int flags);
/* D_c in canonical form: [aggregate][d][row][col] complex128, d = 0 the aggregate itself,
 * d = 1 + 2 mu its forward and d = 2 + 2 mu its backward neighbour in direction mu. On a
 * block grid of extent 2 in direction mu both neighbours are one aggregate and the
 * forward block holds the whole coupling (the backward block is zero). */
int sapdd_mg_coarse_operator(sapdd_mg *mg, double *stencil, int flags);
/* out = the coarse solve of D_c e = rhs (coarse_cycles cycles of GMRES(coarse_iters)
 * from zero) for n canonical coarse vectors; rhs rounded to FP32. */
int sapdd_mg_coarse_solve(sapdd_mg *mg, int n, const double *rhs, double *out, int flags);
/* out = B(in) for nrhs canonical spinors. */
int sapdd_mg_precond(sapdd_mg *mg, int nrhs, const double *in, double *out, int flags);
/* Solve M x = b (the multigrid's kappa) with FGMRES(params->restart) preconditioned by B:
 * the batch solver with the multigrid cycle in place of the plain SAP application, its
 * smoother set by params (nmr, ncy, sap_prec). Same arguments and results as
 * sapdd_solve; the multigrid object keeps the batch for later calls. Near the critical
 * kappa keep ncy small (1-2): every further SAP cycle per application amplifies the
 * slowest modes again (measured: 44 outer steps at ncy 2, no convergence at ncy 5). */
int sapdd_mg_solve(sapdd_mg *mg, const sapdd_params *params, int nrhs, const double *b, double *x,
                   sapdd_stats *stats);
/* Make a batch (no slot in use) precondition with mg instead of SAP; every RHS added
 * later must use mg's kappa. mg must outlive the batch's use of it. */
int sapdd_batch_set_mg(sapdd_batch *batch, sapdd_mg *mg);

/* Bytes of device memory a solve of nrhs RHS with these parameters allocates on top of
 * the resident field (Krylov bases, SAP state, operator copies), for admission control. */
long long sapdd_solve_footprint(const sapdd_field *field, const sapdd_params *params, int nrhs);

/* Device copy of n bytes (STREAM-type copy kernel, used to measure the attainable HBM
 * bandwidth); src and dst are device pointers. */
int sapdd_copy(sapdd_ctx *ctx, const void *src, void *dst, long long n);

/* Per-kernel device time, measured with HIP events recorded on the context's stream
 * around every launch of each kernel family while profiling is on. */
enum {
    SAPDD_K_SAP_HALF = 0,     /* fused gather + MR block solve, one colour           */
    SAPDD_K_DSLASH = 1,       /* full Wilson-clover operator                        */
    SAPDD_K_GS = 2,           /* Gram-Schmidt passes and their reductions            */
    SAPDD_K_BLOCK_DSLASH = 3, /* block-diagonal operator M_B                        */
    SAPDD_K_UPDATE = 4,       /* solution update x += Z y                            */
    SAPDD_K_COPY = 5,         /* bandwidth-probe copy                                */
    SAPDD_K_MG_FINE = 6,      /* multigrid restriction, interpolation and update     */
    SAPDD_K_MG_COARSE = 7,    /* multigrid coarse GMRES                              */
    SAPDD_K_COUNT = 8
};
typedef struct {
    long long launches[SAPDD_K_COUNT];
    double seconds[SAPDD_K_COUNT];
} sapdd_kernel_profile;
/* Read (if out != NULL) and reset the accumulated profile, then switch profiling off
 * (enable = 0), on for every family (enable = 1) or on for the families whose bits are
 * set in enable >> 1 (bit k = family k; few families = fewer event records in flight).
 * Reading waits for the context's stream. */
int sapdd_profile(sapdd_ctx *ctx, int enable, sapdd_kernel_profile *out);

#ifdef __cplusplus
}
#endif
#endif /* SAPDD_H */
