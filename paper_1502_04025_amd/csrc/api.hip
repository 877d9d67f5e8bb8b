// api.hip - the C ABI of include/sapdd.h: contexts, resident fields, the operator and
// preconditioner calls, and the SAP-preconditioned FP64 flexible GMRES driver.
//
// FGMRES(m) (the paper's outer solver without deflation, Sec. 3.1) runs all right-hand
// sides of a call in lock step: one preconditioner launch sequence, one operator launch
// and three Gram-Schmidt passes serve every active RHS. The basis is orthogonalised by
// classical Gram-Schmidt applied twice (CGS2) entirely on the device; the host receives
// only the Hessenberg column (j + 2 complex numbers per RHS) once per step and applies
// the Givens rotations. Every restart recomputes the true residual b - M x in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sapdd.h"
#include "dense.hpp"
#include "kernels.hpp"

using namespace sapdd;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
};

size_t prec_bytes(int prec) { return prec == P64 ? 8 : prec == P32 ? 4 : 2; }
// Storage precisions of a Schwarz mode (sapdd_params.sap_prec): links and clover X, and
// the Schwarz spinors (residual, correction). SAPDD_F16_LINKS keeps the spinors in FP32.
int lprec(int mode) { return mode == SAPDD_F16_LINKS ? P16 : mode; }
int sprec(int mode) { return mode == SAPDD_F16_LINKS ? P32 : mode; }

struct XEntry {  // SAP clover X for one (kappa, precision)
    double kappa;
    int prec;
    Fld x;
    unsigned long long last_use;
    int refs;  // batch slots using it; entries with refs > 0 are never evicted
};

}  // namespace

struct sapdd_field {
    Geom geo;
    double *links64 = nullptr;
    double *tclov64 = nullptr;
    Fld links_lo[3] = {};  // [P32], [P16] lower-precision copies, made on demand
    Fld tclov_lo[3] = {};
    Fld links12[3] = {};   // [P32], [P16] links as their first two rows, made on demand
    std::vector<XEntry> xcache;
    std::vector<Fld> xspare;  // clover buffers of singular kappas, reused by the next one
    unsigned long long use_clock = 0;
    double csw = 0.0;
    // unique per loaded field: a kept batch is reused only for the very field it was
    // built on, never for a later field that happens to get the same address
    unsigned long long id = 0;
};

struct sapdd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::map<std::string, DevBuf> bufs;  // grow-only named workspaces
    int *d_flag = nullptr;
    char *pinned = nullptr;  // host staging for small transfers
    size_t pinned_n = 0;
    hipEvent_t ev[8] = {};
    sapdd_batch *solve_batch = nullptr;  // kept between sapdd_solve calls
    // kernel profiling: event pairs recorded around launches of the selected families
    // (bit k of prof_mask = family k), drained at sync points
    bool prof = false, prof_open = false;
    unsigned prof_mask = 0;
    std::vector<hipEvent_t> pev;
    std::vector<int> pkind, pcount;
    size_t pn = 0;
    long long plaunch[SAPDD_K_COUNT] = {};
    double psec[SAPDD_K_COUNT] = {};
};

namespace {

int fail(sapdd_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(ctx, e_ == hipErrorOutOfMemory ? SAPDD_ENOMEM : SAPDD_EDEVICE, "%s: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                             \
    } while (0)

// Accumulate the elapsed time of every recorded event pair (the stream must have
// completed them) and recycle the pool.
int prof_drain(sapdd_ctx *c) {
    for (size_t i = 0; i < c->pn; ++i) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->pev[2 * i], c->pev[2 * i + 1]));
        c->psec[c->pkind[i]] += ms * 1e-3;
        c->plaunch[c->pkind[i]] += c->pcount[i];
    }
    c->pn = 0;
    return SAPDD_OK;
}

// Record the start event of a profiled launch of family `kind` (no-op when profiling is off).
int prof_begin(sapdd_ctx *c, int kind) {
    c->prof_open = c->prof && (c->prof_mask >> kind & 1u);
    if (!c->prof_open) return SAPDD_OK;
    if (2 * (c->pn + 1) > c->pev.size()) {
        if (c->pev.size() >= 8192) {  // pool full: wait for the stream and drain it
            HIPCHK(c, hipStreamSynchronize(c->stream));
            int r = prof_drain(c);
            if (r != SAPDD_OK) return r;
        } else {
            const size_t old = c->pev.size();
            c->pev.resize(old ? 2 * old : 256);
            c->pkind.resize(c->pev.size() / 2);
            c->pcount.resize(c->pev.size() / 2);
            for (size_t i = old; i < c->pev.size(); ++i) HIPCHK(c, hipEventCreate(&c->pev[i]));
        }
    }
    c->pkind[c->pn] = kind;
    c->pcount[c->pn] = 1;
    HIPCHK(c, hipEventRecord(c->pev[2 * c->pn], c->stream));
    return SAPDD_OK;
}

// End a profiled region that contained `count` launches of its family (a graph replay).
int prof_end(sapdd_ctx *c, int count = 1) {
    if (!c->prof_open) return SAPDD_OK;
    c->prof_open = false;
    c->pcount[c->pn] = count;
    HIPCHK(c, hipEventRecord(c->pev[2 * c->pn + 1], c->stream));
    c->pn += 1;
    return SAPDD_OK;
}

#define CHK(expr)             \
    do {                      \
        int r_ = (expr);      \
        if (r_ != SAPDD_OK) return r_; \
    } while (0)

// A kernel launch timed under profiling.
#define KLAUNCH(ctx, kind, call)            \
    do {                                    \
        CHK(prof_begin(ctx, kind));         \
        HIPCHK(ctx, call);                  \
        CHK(prof_end(ctx));                 \
    } while (0)

// Named grow-only device buffer.
int buf(sapdd_ctx *c, const char *name, size_t bytes, void **out) {
    DevBuf &b = c->bufs[name];
    if (b.n < bytes) {
        if (b.p) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            HIPCHK(c, hipFree(b.p));
            b.p = nullptr;
            b.n = 0;
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, SAPDD_ENOMEM, "hipMalloc of %zu bytes for %s failed", bytes, name);
        }
        b.p = p;
        b.n = bytes;
    }
    *out = b.p;
    return SAPDD_OK;
}

int pinned(sapdd_ctx *c, size_t bytes, void **out) {
    if (c->pinned_n < bytes) {
        if (c->pinned) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            HIPCHK(c, hipHostFree(c->pinned));
            c->pinned = nullptr;
        }
        HIPCHK(c, hipHostMalloc((void **)&c->pinned, bytes, hipHostMallocDefault));
        c->pinned_n = bytes;
    }
    *out = c->pinned;
    return SAPDD_OK;
}

// A spinor-shaped field of nf copies in precision prec inside buffer `name`.
int spinor_buf(sapdd_ctx *c, const char *name, const Geom &g, int nf, int prec, int ncomp, Fld *f) {
    const size_t nd = (size_t)g.V * ncomp * nf;
    size_t bytes = nd * prec_bytes(prec);
    const size_t sc_off = (bytes + 255) / 256 * 256;
    if (prec == P16) bytes = sc_off + (size_t)g.V * nf * sizeof(float);
    void *p;
    CHK(buf(c, name, bytes, &p));
    f->data = p;
    f->scale = prec == P16 ? (float *)((char *)p + sc_off) : nullptr;
    f->prec = prec;
    return SAPDD_OK;
}

bool supported_block(const int b[4]) {
    return (b[0] == 2 && b[1] == 2 && b[2] == 2 && b[3] == 2) || (b[0] == 4 && b[1] == 4 && b[2] == 4 && b[3] == 4) ||
           (b[0] == 8 && b[1] == 4 && b[2] == 4 && b[3] == 4);
}

// Host->device staging of a canonical array (or pass-through of a device pointer).
int stage_in(sapdd_ctx *c, const char *name, const double *p, size_t ndouble, int flags, const double **out) {
    if (flags & SAPDD_DEVICE_PTRS) {
        *out = p;
        return SAPDD_OK;
    }
    void *d;
    CHK(buf(c, name, ndouble * 8, &d));
    HIPCHK(c, hipMemcpyAsync(d, p, ndouble * 8, hipMemcpyHostToDevice, c->stream));
    *out = (const double *)d;
    return SAPDD_OK;
}

int lo_copies(sapdd_ctx *c, sapdd_field *f, int prec) {
    if (prec == P64 || f->links_lo[prec].data) return SAPDD_OK;
    const Geom &g = f->geo;
    for (int which = 0; which < 2; ++which) {
        Fld fl;
        size_t bytes = (size_t)g.V * 72 * prec_bytes(prec);
        const size_t sc_off = (bytes + 255) / 256 * 256;
        if (prec == P16) bytes = sc_off + (size_t)g.V * sizeof(float);
        void *p = nullptr;
        HIPCHK(c, hipMalloc(&p, bytes));
        fl.data = p;
        fl.scale = prec == P16 ? (float *)((char *)p + sc_off) : nullptr;
        fl.prec = prec;
        HIPCHK(c, launch_convert(g, 72, 1, which == 0 ? f->links64 : f->tclov64, fl, c->stream));
        (which == 0 ? f->links_lo[prec] : f->tclov_lo[prec]) = fl;
    }
    return SAPDD_OK;
}

// The links as their first two rows in storage precision prec (P32 or P16), made once.
int links12_copy(sapdd_ctx *c, sapdd_field *f, int prec) {
    if (f->links12[prec].data) return SAPDD_OK;
    const Geom &g = f->geo;
    size_t bytes = (size_t)g.V * 48 * prec_bytes(prec);
    const size_t sc_off = (bytes + 255) / 256 * 256;
    if (prec == P16) bytes = sc_off + (size_t)g.V * sizeof(float);
    void *p = nullptr;
    HIPCHK(c, hipMalloc(&p, bytes));
    Fld fl{p, prec == P16 ? (float *)((char *)p + sc_off) : nullptr, prec};
    HIPCHK(c, launch_links12_pack(g, f->links64, fl, c->stream));
    f->links12[prec] = fl;
    return SAPDD_OK;
}

Fld links_of(const sapdd_field *f, int prec) {
    if (prec == P64) return Fld{f->links64, nullptr, P64};
    return f->links_lo[prec];
}
Fld tclov_of(const sapdd_field *f, int prec) {
    if (prec == P64) return Fld{f->tclov64, nullptr, P64};
    return f->tclov_lo[prec];
}

void free_fld(Fld &x) {
    if (x.data) (void)hipFree(x.data);
    x = Fld{};
}

constexpr size_t XCACHE_ENTRIES = 16;

// Gram-Schmidt: the second correction is skipped where |c|^2 <= CGS_SKIP_TOL |w'|^2.
constexpr double CGS_SKIP_TOL = 1e-18;

int clover_buffer(sapdd_ctx *c, const Geom &g, int prec, Fld *x) {
    size_t bytes = (size_t)g.V * 72 * prec_bytes(prec);
    const size_t sc_off = (bytes + 255) / 256 * 256;
    if (prec == P16) bytes = sc_off + (size_t)g.V * sizeof(float);
    void *p = nullptr;
    HIPCHK(c, hipMalloc(&p, bytes));
    *x = Fld{p, prec == P16 ? (float *)((char *)p + sc_off) : nullptr, prec};
    return SAPDD_OK;
}

// Allocate now the buffers the field's clover cache can hold in this precision (spares
// that the next kappas fill), so that admitting a kappa later allocates nothing.
int reserve_clover_cache(sapdd_ctx *c, sapdd_field *f, int prec) {
    size_t have = 0;
    for (auto &e : f->xcache) have += e.prec == prec;
    for (auto &x : f->xspare) have += x.prec == prec;
    for (; have < XCACHE_ENTRIES; ++have) {
        Fld x{};
        CHK(clover_buffer(c, f->geo, prec, &x));
        f->xspare.push_back(x);
    }
    return SAPDD_OK;
}

// SAP clover X for (kappa, prec), cached on the field: at most 16 entries. A new kappa
// fills a spare buffer (reserve_clover_cache, or one a singular kappa left), else
// recomputes into the buffer of the least recently used unreferenced entry, rather than
// freeing one: hipFree waits for the whole device, the other
// streams' work included, which stalled concurrent serving volumes for the length of
// their steps. `ref` adds a reference that sap_clover_release drops.
int sap_clover(sapdd_ctx *c, sapdd_field *f, double kappa, int prec, Fld *out, bool ref = false) {
    for (auto &e : f->xcache)
        if (e.kappa == kappa && e.prec == prec) {
            e.last_use = ++f->use_clock;
            e.refs += ref ? 1 : 0;
            *out = e.x;
            return SAPDD_OK;
        }
    const size_t max_entries = XCACHE_ENTRIES;
    Fld x{};
    for (size_t i = 0; i < f->xspare.size(); ++i)
        if (f->xspare[i].prec == prec) {
            x = f->xspare[i];
            f->xspare.erase(f->xspare.begin() + i);
            break;
        }
    while (f->xcache.size() >= max_entries) {
        auto it = f->xcache.end();
        for (auto q = f->xcache.begin(); q != f->xcache.end(); ++q)
            if (q->refs == 0 && (it == f->xcache.end() || q->last_use < it->last_use)) it = q;
        if (it == f->xcache.end()) break;  // every entry in use: grow instead
        // the stream's earlier launches may still read the evicted entry; the new
        // kappa's kernel below runs after them on the same stream
        if (!x.data && it->prec == prec) {
            x = it->x;
        } else {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            free_fld(it->x);
        }
        f->xcache.erase(it);
    }
    const Geom &g = f->geo;
    if (!x.data) CHK(clover_buffer(c, g, prec, &x));
    XEntry e;
    e.kappa = kappa;
    e.prec = prec;
    e.last_use = ++f->use_clock;
    e.refs = ref ? 1 : 0;
    e.x = x;
    HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    HIPCHK(c, launch_sap_clover(g, f->tclov64, kappa, e.x, c->d_flag, c->stream));
    int sing = 0;
    HIPCHK(c, hipMemcpyAsync(&sing, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (sing) {
        f->xspare.push_back(x);  // kept for the next kappa
        return fail(c, SAPDD_ESINGULAR, "clover block 1 + kappa T is singular at kappa = %g", kappa);
    }
    f->xcache.push_back(e);
    *out = e.x;
    return SAPDD_OK;
}

void sap_clover_release(sapdd_field *f, double kappa, int prec) {
    for (auto &e : f->xcache)
        if (e.kappa == kappa && e.prec == prec && e.refs > 0) {
            e.refs -= 1;
            return;
        }
}

int check_params(sapdd_ctx *c, const sapdd_field *f, const sapdd_params *p) {
    if (!p) return fail(c, SAPDD_EINVAL, "params is NULL");
    const bool zero = !p->block[0] && !p->block[1] && !p->block[2] && !p->block[3];
    if (!zero)
        for (int mu = 0; mu < 4; ++mu)
            if (p->block[mu] != f->geo.B[mu])
                return fail(c, SAPDD_EINVAL, "params.block differs from the field's blocking");
    if (p->nmr < 1 || p->ncy < 1) return fail(c, SAPDD_EINVAL, "nmr and ncy must be >= 1");
    if (p->sap_prec < SAPDD_F64 || p->sap_prec > SAPDD_F16_LINKS) return fail(c, SAPDD_EINVAL, "bad sap_prec");
    if (!(p->gap >= 0)) return fail(c, SAPDD_EINVAL, "gap must be >= 0 (0 = the default 10)");
    return SAPDD_OK;
}

// Buffers of one preconditioner application for nrhs right-hand sides.
struct SapState {
    Fld links;
    Fld rres, delta;
    const void **X;  // device pointer arrays
    const float **Xsc;
    double *kappa;
};

// Upload per-rhs kappa and clover pointers; prepare rres/delta buffers (mode: sap_prec).
int sap_prepare(sapdd_ctx *c, sapdd_field *f, const double *kappa, int nrhs, int mode, SapState *s) {
    const Geom &g = f->geo;
    const int lp = lprec(mode), sp = sprec(mode);
    CHK(lo_copies(c, f, lp));
    s->links = links_of(f, lp);
    std::vector<Fld> xs(nrhs);
    // referenced while the list is built, so a later kappa of this call never recycles
    // the buffer of an earlier one (more than 16 distinct kappas grow the cache)
    int rc = SAPDD_OK, got = 0;
    for (; got < nrhs && rc == SAPDD_OK; ++got) rc = sap_clover(c, f, kappa[got], lp, &xs[got], true);
    for (int r = 0; r < got - (rc != SAPDD_OK); ++r) sap_clover_release(f, kappa[r], lp);
    CHK(rc);
    CHK(spinor_buf(c, "sap_rres", g, nrhs, sp, 12, &s->rres));
    CHK(spinor_buf(c, "sap_delta", g, nrhs, sp, 24, &s->delta));
    // rres scales are indexed per half lattice: spinor_buf allotted V per field, enough.
    void *meta;
    const size_t mbytes = (size_t)nrhs * (2 * sizeof(void *) + sizeof(double));
    CHK(buf(c, "sap_meta", mbytes, &meta));
    void *host;
    CHK(pinned(c, mbytes, &host));
    HIPCHK(c, hipStreamSynchronize(c->stream));  // the pinned block may still feed a copy
    char *h = (char *)host;
    for (int r = 0; r < nrhs; ++r) {
        ((const void **)h)[r] = xs[r].data;
        ((const float **)(h + nrhs * sizeof(void *)))[r] = xs[r].scale;
        ((double *)(h + 2 * nrhs * sizeof(void *)))[r] = kappa[r];
    }
    HIPCHK(c, hipMemcpyAsync(meta, host, mbytes, hipMemcpyHostToDevice, c->stream));
    s->X = (const void **)meta;
    s->Xsc = (const float **)((char *)meta + nrhs * sizeof(void *));
    s->kappa = (double *)((char *)meta + 2 * nrhs * sizeof(void *));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SAPDD_OK;
}

// Enqueue one SAP application: psi = SAP(eta) for the nact slots.
int sap_run(sapdd_ctx *c, const Geom &g, const SapState &s, const sapdd_params *p, const double *eta, int eta_stride,
            const double *eta_scale, int eta_scale_stride, void *psi, int psi_prec, int psi_stride, const int *active,
            int nact) {
    SapArgsHost a;
    a.links = s.links;
    a.X = s.X;
    a.Xsc = s.links.prec == P16 ? s.Xsc : nullptr;
    a.kappa = s.kappa;
    a.eta = eta;
    a.eta_scale = eta_scale;
    a.eta_scale_stride = eta_scale_stride;
    a.eta_stride_rhs = eta_stride;
    a.rres = s.rres;
    a.delta = s.delta;
    a.psi = psi;
    a.psi_prec = psi_prec;
    a.psi_stride_rhs = psi_stride;
    a.active = active;
    a.nact = nact;
    a.nmr = p->nmr;
    for (int k = 0; k < p->ncy; ++k)
        for (int col = 0; col < 2; ++col) {
            const int mode = k == 0 ? col : 2;
            const int last = (k == p->ncy - 1) && col == 1;
            KLAUNCH(c, SAPDD_K_SAP_HALF, launch_sap_half(g, a, col, mode, !last, c->stream));
        }
    return SAPDD_OK;
}

int identity_list(sapdd_ctx *c, int n, int **out) {
    void *d;
    CHK(buf(c, "ident", (size_t)n * sizeof(int), &d));
    void *h;
    CHK(pinned(c, (size_t)n * sizeof(int), &h));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < n; ++i) ((int *)h)[i] = i;
    HIPCHK(c, hipMemcpyAsync(d, h, (size_t)n * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *out = (int *)d;
    return SAPDD_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ====================================================================== allocation-free SAP
// Device memory for sapdd_sap_noalloc: a file-scope array each GPU holds until the process
// ends. Host code never uses its name as an address (that is a host-side stand-in): the
// device address of every GPU's copy is taken once with hipGetSymbolAddress, with that
// device current, and kept in noalloc_ptr[device].
#define SAPDD_NOALLOC_BYTES (256ull << 20)
#define SAPDD_NOALLOC_MAX_RHS 16
static __device__ __align__(256) unsigned char scratch[SAPDD_NOALLOC_BYTES];

namespace {

std::mutex noalloc_mu;
void *noalloc_ptr[64] = {};
int noalloc_status[64] = {};  // 0 not looked up, 1 ok, -1 lookup failed

// Look up this device's scratch address (the device must be current).
int noalloc_setup(int device) {
    if (device < 0 || device >= 64) return SAPDD_EDEVICE;
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (noalloc_status[device] == 0) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e == hipSuccess && ptr) {
            noalloc_ptr[device] = ptr;
            noalloc_status[device] = 1;
        } else {
            (void)hipGetLastError();
            noalloc_status[device] = -1;
        }
    }
    return noalloc_status[device] == 1 ? SAPDD_OK : SAPDD_EDEVICE;
}

struct NoallocMeta {
    const void *X[SAPDD_NOALLOC_MAX_RHS];
    const float *Xsc[SAPDD_NOALLOC_MAX_RHS];
    double kappa[SAPDD_NOALLOC_MAX_RHS];
    int n;
};

__global__ void set_int_kernel(int *p, int v) { *p = v; }

// Zero n doubles (n even). A kernel rather than hipMemsetAsync: an elastic slot's range
// spans several mappings, which the runtime's memset rejects.
__global__ void zero_kernel(double2 *p, int64_t n2) {
    const double2 z = make_double2(0.0, 0.0);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z;
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t st) {
    const int64_t n2 = n / 2;
    const int64_t blocks = std::min<int64_t>((n2 + 255) / 256, 65536);
    if (blocks > 0) hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (double2 *)p, n2);
    return hipGetLastError();
}

// One slot's clover pointers and kappa for the batch kernels, passed as kernel arguments
// (no host staging buffer that a later add could overwrite before the copy ran).
__global__ void slot_meta_kernel(const void **X, const float **Xsc, double *kappa, int r, const void *x,
                                 const float *xs, double k) {
    X[r] = x;
    Xsc[r] = xs;
    kappa[r] = k;
}

// Writes the per-rhs clover pointers, kappa and the identity slot list into the scratch
// memory and clears the singular-pivot flag (a kernel, not a memset).
__global__ void noalloc_meta_kernel(NoallocMeta m, const void **X, const float **Xsc, double *kappa, int *ident,
                                    int *flag) {
    const int i = threadIdx.x;
    if (i < m.n) {
        X[i] = m.X[i];
        Xsc[i] = m.Xsc[i];
        kappa[i] = m.kappa[i];
        ident[i] = i;
    }
    if (i == 0) *flag = 0;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int sapdd_create(int device, void *hip_stream, sapdd_ctx **out) {
    if (!out) return SAPDD_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SAPDD_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return SAPDD_EDEVICE;
    sapdd_ctx *c = new sapdd_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipMalloc((void **)&c->d_flag, 256) != hipSuccess) {
        delete c;
        return SAPDD_ENOMEM;
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete c;
            return SAPDD_EDEVICE;
        }
    // the allocation-free entry point's memory on this device (a failed lookup only
    // disables that entry point, which then reports it)
    (void)noalloc_setup(device);
    *out = c;
    return SAPDD_OK;
}

void sapdd_destroy(sapdd_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->solve_batch) sapdd_batch_destroy(c->solve_batch);
    for (auto &kv : c->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (c->d_flag) (void)hipFree(c->d_flag);
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->pev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

const char *sapdd_last_error(const sapdd_ctx *c) { return c ? c->err.c_str() : "null context"; }

int sapdd_load_gauge(sapdd_ctx *c, const int dims[4], const int block[4], const double *links, int antiperiodic_t,
                     int flags, sapdd_field **out) {
    if (!c || !dims || !block || !links || !out) return fail(c, SAPDD_EINVAL, "null argument");
    *out = nullptr;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    if (!supported_block(block))
        return fail(c, SAPDD_EINVAL, "unsupported block %dx%dx%dx%d (2x2x2x2, 4x4x4x4 or 8x4x4x4)", block[0], block[1],
                    block[2], block[3]);
    Geom g;
    g.V = 1;
    g.Nd = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] <= 0 || dims[mu] % block[mu])
            return fail(c, SAPDD_EINVAL, "block extent %d does not divide lattice extent %d", block[mu], dims[mu]);
        if ((dims[mu] / block[mu]) % 2)
            return fail(c, SAPDD_EINVAL, "the block grid must be even in every direction (two-colouring)");
        g.L[mu] = dims[mu];
        g.B[mu] = block[mu];
        g.G[mu] = dims[mu] / block[mu];
        g.V *= dims[mu];
        g.Nd *= g.G[mu];
    }
    g.Vb = block[0] * block[1] * block[2] * block[3];
    g.Vbh = g.Vb / 2;
    g.antiperiodic = antiperiodic_t ? 1 : 0;
    if ((g.Nd / 2) > 0x7fffffffLL || g.V * 24 > (1LL << 40)) return fail(c, SAPDD_EINVAL, "lattice too large");
    sapdd_field *f = new sapdd_field;
    // fields may be loaded from several host threads (one context each)
    static std::atomic<unsigned long long> next_field_id{0};
    f->id = next_field_id.fetch_add(1) + 1;
    f->geo = g;
    hipError_t e1 = hipMalloc((void **)&f->links64, (size_t)g.V * 72 * 8);
    hipError_t e2 = e1 == hipSuccess ? hipMalloc((void **)&f->tclov64, (size_t)g.V * 72 * 8) : e1;
    if (e2 != hipSuccess) {
        if (f->links64) (void)hipFree(f->links64);
        delete f;
        (void)hipGetLastError();
        return fail(c, SAPDD_ENOMEM, "cannot allocate the gauge field");
    }
    const double *src;
    int r = stage_in(c, "stage_in", links, (size_t)g.V * 72, flags, &src);
    if (r == SAPDD_OK) {
        hipError_t e = launch_pack(g, 72, 1, src, Fld{f->links64, nullptr, P64}, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(f->tclov64, 0, (size_t)g.V * 72 * 8, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) r = fail(c, SAPDD_EDEVICE, "load_gauge: %s", hipGetErrorString(e));
    }
    if (r != SAPDD_OK) {
        sapdd_free_field(c, f);
        return r;
    }
    *out = f;
    return SAPDD_OK;
}

static void drop_derived(sapdd_field *f) {
    for (int p = 1; p < 3; ++p) {
        free_fld(f->links_lo[p]);
        free_fld(f->tclov_lo[p]);
        free_fld(f->links12[p]);
    }
    for (auto &e : f->xcache) free_fld(e.x);
    f->xcache.clear();
    for (auto &x : f->xspare) free_fld(x);
    f->xspare.clear();
}

int sapdd_compute_clover(sapdd_ctx *c, sapdd_field *f, double csw) {
    if (!c || !f) return fail(c, SAPDD_EINVAL, "null argument");
    if (!(csw >= 0.0)) return fail(c, SAPDD_EINVAL, "c_sw must be >= 0");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_derived(f);
    HIPCHK(c, launch_clover_build(f->geo, f->links64, csw, f->tclov64, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    f->csw = csw;
    return SAPDD_OK;
}

int sapdd_load_clover(sapdd_ctx *c, sapdd_field *f, const double *clover, int flags) {
    if (!c || !f || !clover) return fail(c, SAPDD_EINVAL, "null argument");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_derived(f);
    const double *src;
    CHK(stage_in(c, "stage_in", clover, (size_t)f->geo.V * 288, flags, &src));
    HIPCHK(c, launch_clover_pack(f->geo, src, f->tclov64, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SAPDD_OK;
}

}  // extern "C"
static const sapdd_field *batch_field(const sapdd_batch *B);
extern "C" {

int sapdd_free_field(sapdd_ctx *c, sapdd_field *f) {
    if (!f) return SAPDD_OK;
    if (c) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
    }
    if (c && c->solve_batch && batch_field(c->solve_batch) == f) {  // the kept batch holds this field's buffers
        sapdd_batch_destroy(c->solve_batch);
        c->solve_batch = nullptr;
    }
    drop_derived(f);
    if (f->links64) (void)hipFree(f->links64);
    if (f->tclov64) (void)hipFree(f->tclov64);
    delete f;
    return SAPDD_OK;
}

static int apply_common(sapdd_ctx *c, const sapdd_field *fc, double kappa, int prec, int nrhs, const double *in,
                        double *out, int flags, bool block) {
    if (!c || !fc || !in || !out) return fail(c, SAPDD_EINVAL, "null argument");
    if (nrhs < 1) return fail(c, SAPDD_EINVAL, "nrhs must be >= 1");
    if (prec < SAPDD_F64 || prec > SAPDD_F16) return fail(c, SAPDD_EINVAL, "bad precision");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_field *f = const_cast<sapdd_field *>(fc);
    const Geom &g = f->geo;
    const size_t nd = (size_t)g.V * 24 * nrhs;
    const bool two_row = block && (flags & SAPDD_LINKS12);
    if (two_row && prec == P64) return fail(c, SAPDD_EINVAL, "two-row links are for FP32 and FP16 storage");
    CHK(lo_copies(c, f, prec));
    if (two_row) CHK(links12_copy(c, f, prec));
    const double *src;
    CHK(stage_in(c, "stage_in", in, nd, flags, &src));
    Fld fin, fout;
    CHK(spinor_buf(c, "op_in", g, nrhs, prec, 24, &fin));
    CHK(spinor_buf(c, "op_out", g, nrhs, prec, 24, &fout));
    HIPCHK(c, launch_pack(g, 24, nrhs, src, fin, c->stream));
    if (two_row) {
        KLAUNCH(c, SAPDD_K_BLOCK_DSLASH,
                launch_dslash_block12(g, f->links12[prec], tclov_of(f, prec), kappa, fin, fout, nrhs, c->stream));
    } else if (block) {
        KLAUNCH(c, SAPDD_K_BLOCK_DSLASH, launch_dslash_block(g, links_of(f, prec), tclov_of(f, prec), kappa, fin, fout, nrhs, c->stream));
    } else {
        int *ident;
        CHK(identity_list(c, nrhs, &ident));
        DslashIO io{};
        io.in = fin;
        io.out = fout;
        io.active = ident;
        io.nact = nrhs;
        io.in_stride = io.out_stride = io.sub_stride = 1;
        KLAUNCH(c, SAPDD_K_DSLASH, launch_dslash_full(g, links_of(f, prec), tclov_of(f, prec), kappa, io, c->stream));
    }
    double *dst = out;
    if (!(flags & SAPDD_DEVICE_PTRS)) {
        void *d;
        CHK(buf(c, "stage_out", nd * 8, &d));
        dst = (double *)d;
    }
    HIPCHK(c, launch_unpack(g, 24, nrhs, fout, dst, c->stream));
    if (!(flags & SAPDD_DEVICE_PTRS)) HIPCHK(c, hipMemcpyAsync(out, dst, nd * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SAPDD_OK;
}

int sapdd_apply_D(sapdd_ctx *c, const sapdd_field *f, double kappa, int prec, int nrhs, const double *in, double *out,
                  int flags) {
    return apply_common(c, f, kappa, prec, nrhs, in, out, flags, false);
}

int sapdd_apply_block_D(sapdd_ctx *c, const sapdd_field *f, double kappa, int prec, int nrhs, const double *in,
                        double *out, int flags) {
    return apply_common(c, f, kappa, prec, nrhs, in, out, flags, true);
}

int sapdd_sap(sapdd_ctx *c, const sapdd_field *fc, const double *kappa, const sapdd_params *p, int nrhs,
              const double *in, double *out) {
    if (!c || !fc || !kappa || !in || !out) return fail(c, SAPDD_EINVAL, "null argument");
    if (nrhs < 1) return fail(c, SAPDD_EINVAL, "nrhs must be >= 1");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_field *f = const_cast<sapdd_field *>(fc);
    CHK(check_params(c, f, p));
    const Geom &g = f->geo;
    const size_t nd = (size_t)g.V * 24 * nrhs;
    const int prec = p->sap_prec;
    const int psi_prec = prec == P64 ? P64 : P32;
    for (int r = 0; r < nrhs; ++r)
        if (!(kappa[r] > 0)) return fail(c, SAPDD_EINVAL, "kappa must be > 0");
    SapState s;
    CHK(sap_prepare(c, f, kappa, nrhs, prec, &s));
    const double *src;
    CHK(stage_in(c, "stage_in", in, nd, p->flags, &src));
    Fld eta, psi;
    CHK(spinor_buf(c, "sap_eta", g, nrhs, P64, 24, &eta));
    CHK(spinor_buf(c, "sap_psi", g, nrhs, psi_prec, 24, &psi));
    HIPCHK(c, launch_pack(g, 24, nrhs, src, eta, c->stream));
    int *ident;
    CHK(identity_list(c, nrhs, &ident));
    CHK(sap_run(c, g, s, p, (const double *)eta.data, 1, nullptr, 0, psi.data, psi_prec, 1, ident, nrhs));
    double *dst = out;
    if (!(p->flags & SAPDD_DEVICE_PTRS)) {
        void *d;
        CHK(buf(c, "stage_out", nd * 8, &d));
        dst = (double *)d;
    }
    HIPCHK(c, launch_unpack(g, 24, nrhs, psi, dst, c->stream));
    if (!(p->flags & SAPDD_DEVICE_PTRS)) HIPCHK(c, hipMemcpyAsync(out, dst, nd * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SAPDD_OK;
}

int sapdd_sap_noalloc(sapdd_ctx *c, const sapdd_field *fc, const double *kappa, const sapdd_params *p, int nrhs,
                      const double *in, double *out) {
    if (!c || !fc || !kappa || !in || !out) return fail(c, SAPDD_EINVAL, "null argument");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    const sapdd_field *f = fc;
    CHK(check_params(c, f, p));
    if (!(p->flags & SAPDD_DEVICE_PTRS))
        return fail(c, SAPDD_EINVAL, "sapdd_sap_noalloc takes device pointers only (SAPDD_DEVICE_PTRS)");
    if (nrhs < 1 || nrhs > SAPDD_NOALLOC_MAX_RHS)
        return fail(c, SAPDD_EINVAL, "sapdd_sap_noalloc takes 1..%d right-hand sides", SAPDD_NOALLOC_MAX_RHS);
    for (int r = 0; r < nrhs; ++r)
        if (!(kappa[r] > 0)) return fail(c, SAPDD_EINVAL, "kappa must be > 0");
    if (noalloc_setup(c->device) != SAPDD_OK)
        return fail(c, SAPDD_EDEVICE, "the scratch memory of device %d has no device address", c->device);
    const Geom &g = f->geo;
    const int prec = p->sap_prec, lp = lprec(prec), sp = sprec(prec);
    const int psi_prec = prec == P64 ? P64 : P32;
    const size_t V = (size_t)g.V;
    auto al = [](size_t n) { return (n + 255) / 256 * 256; };
    auto fld_bytes = [&](size_t ncomp, size_t nf, int pr) {  // data, then FP16 scales (V per field)
        const size_t d = al(V * ncomp * nf * prec_bytes(pr));
        return pr == P16 ? d + al(V * nf * sizeof(float)) : d;
    };
    // distinct kappa values get one clover X each (fixed-size host arrays: nothing here
    // allocates, on the device or on the host)
    double kv[SAPDD_NOALLOC_MAX_RHS];
    int kidx[SAPDD_NOALLOC_MAX_RHS], nk = 0;
    for (int r = 0; r < nrhs; ++r) {
        int q = 0;
        while (q < nk && kv[q] != kappa[r]) ++q;
        if (q == nk) kv[nk++] = kappa[r];
        kidx[r] = q;
    }
    const bool need_links = lp != P64 && !f->links_lo[lp].data;
    const size_t off_meta = 256;
    const size_t meta_bytes = al(nrhs * (2 * sizeof(void *) + sizeof(double) + sizeof(int)));
    const size_t off_x = off_meta + meta_bytes;
    const size_t x_bytes = fld_bytes(72, 1, lp);
    const size_t off_links = off_x + nk * x_bytes;
    const size_t off_eta = off_links + (need_links ? fld_bytes(72, 1, lp) : 0);
    const size_t off_psi = off_eta + fld_bytes(24, nrhs, P64);
    const size_t off_rres = off_psi + fld_bytes(24, nrhs, psi_prec);
    const size_t off_delta = off_rres + fld_bytes(12, nrhs, sp);
    const size_t total = off_delta + fld_bytes(24, nrhs, sp);
    if (total > SAPDD_NOALLOC_BYTES)
        return fail(c, SAPDD_EINVAL,
                    "sapdd_sap_noalloc needs %zu bytes of scratch for this lattice, precision and %d right-hand "
                    "sides; its fixed maximum is %llu",
                    total, nrhs, (unsigned long long)SAPDD_NOALLOC_BYTES);
    char *base = (char *)noalloc_ptr[c->device];
    auto fld = [&](size_t off, size_t ncomp, size_t nf, int pr) {
        return Fld{base + off, pr == P16 ? (float *)(base + off + al(V * ncomp * nf * prec_bytes(pr))) : nullptr, pr};
    };
    int *flag = (int *)base;
    const void **dX = (const void **)(base + off_meta);
    const float **dXsc = (const float **)(base + off_meta + nrhs * sizeof(void *));
    double *dk = (double *)(base + off_meta + 2 * nrhs * sizeof(void *));
    int *ident = (int *)(base + off_meta + 2 * nrhs * sizeof(void *) + nrhs * sizeof(double));
    // clover X per distinct kappa (singular pivots flagged), low-precision links if the
    // field has none yet, per-rhs metadata
    NoallocMeta m{};
    m.n = nrhs;
    Fld xs[SAPDD_NOALLOC_MAX_RHS];
    for (int q = 0; q < nk; ++q) xs[q] = fld(off_x + q * x_bytes, 72, 1, lp);
    for (int r = 0; r < nrhs; ++r) {
        m.X[r] = xs[kidx[r]].data;
        m.Xsc[r] = xs[kidx[r]].scale;
        m.kappa[r] = kappa[r];
    }
    hipLaunchKernelGGL(noalloc_meta_kernel, dim3(1), dim3(64), 0, c->stream, m, dX, dXsc, dk, ident, flag);
    HIPCHK(c, hipGetLastError());
    for (int q = 0; q < nk; ++q) HIPCHK(c, launch_sap_clover(g, f->tclov64, kv[q], xs[q], flag, c->stream));
    SapState s;
    if (lp == P64) {
        s.links = Fld{f->links64, nullptr, P64};
    } else if (need_links) {
        s.links = fld(off_links, 72, 1, lp);
        HIPCHK(c, launch_convert(g, 72, 1, f->links64, s.links, c->stream));
    } else {
        s.links = f->links_lo[lp];
    }
    s.rres = fld(off_rres, 12, nrhs, sp);
    s.delta = fld(off_delta, 24, nrhs, sp);
    s.X = dX;
    s.Xsc = dXsc;
    s.kappa = dk;
    const Fld eta = fld(off_eta, 24, nrhs, P64), psi = fld(off_psi, 24, nrhs, psi_prec);
    HIPCHK(c, launch_pack(g, 24, nrhs, in, eta, c->stream));
    // the kernel profiler's event pool may grow: it stays off inside this call
    const bool prof = c->prof;
    c->prof = false;
    const int rs = sap_run(c, g, s, p, (const double *)eta.data, 1, nullptr, 0, psi.data, psi_prec, 1, ident, nrhs);
    c->prof = prof;
    CHK(rs);
    HIPCHK(c, launch_unpack(g, 24, nrhs, psi, out, c->stream));
    int sing = 0;
    HIPCHK(c, hipMemcpyAsync(&sing, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (sing) return fail(c, SAPDD_ESINGULAR, "clover block 1 + kappa T is singular for one of the kappa values");
    return SAPDD_OK;
}

long long sapdd_solve_footprint(const sapdd_field *f, const sapdd_params *p, int nrhs) {
    if (!f || !p || nrhs < 1) return -1;
    const long long V = f->geo.V;
    const int m = std::max(1, p->restart);
    const int prec = p->sap_prec, lp = lprec(prec), sp = sprec(prec);
    const long long lb = (long long)prec_bytes(lp), sb = (long long)prec_bytes(sp);
    const long long zb = prec == P64 || p->deflate > 0 ? 8 : 4;
    long long per_rhs = (m + 1) * V * 24 * 8     // Krylov basis V
                        + (long long)m * V * 24 * zb  // preconditioned vectors Z
                        + 2 * V * 24 * 8              // b and x in the device layout
                        + V * 24 * sb + V * 12 * sb + (sp == P16 ? 2 * V * 4 : 0)  // SAP delta, residual
                        + V * 72 * lb + (lp == P16 ? V * 4 : 0);                    // clover X per kappa
    long long fixed = lp == P64 ? 0 : 2 * V * 72 * lb + (lp == P16 ? 2 * V * 4 : 0);  // low-precision links, T
    return fixed + per_rhs * nrhs;
}

int sapdd_profile(sapdd_ctx *c, int enable, sapdd_kernel_profile *out) {
    if (!c) return SAPDD_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    CHK(prof_drain(c));
    if (out)
        for (int k = 0; k < SAPDD_K_COUNT; ++k) {
            out->launches[k] = c->plaunch[k];
            out->seconds[k] = c->psec[k];
        }
    for (int k = 0; k < SAPDD_K_COUNT; ++k) {
        c->plaunch[k] = 0;
        c->psec[k] = 0;
    }
    c->prof = enable != 0;
    c->prof_mask = enable == 1 ? ~0u : (unsigned)enable >> 1;
    return SAPDD_OK;
}

int sapdd_copy(sapdd_ctx *c, const void *src, void *dst, long long n) {
    if (!c || !src || !dst || n < 0) return fail(c, SAPDD_EINVAL, "bad copy arguments");
    HIPCHK(c, hipSetDevice(c->device));
    KLAUNCH(c, SAPDD_K_COPY, launch_copy(src, dst, n, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SAPDD_OK;
}

}  // extern "C"


// ====================================================================== multigrid state
// The two-level preconditioner (Sec. 2.6: a Krylov solver preconditioned by a multigrid
// cycle whose smoother is the Schwarz procedure). P and D_c are resident; every
// application runs restriction, the coarse GMRES, interpolation, the FP64 residual, the
// SAP smoother and the update as one launch sequence over the listed systems.
struct sapdd_mg {
    sapdd_ctx *c = nullptr;
    sapdd_field *f = nullptr;
    double kappa = 0;
    sapdd_params sp{};     // smoother of the set-up and of sapdd_mg_precond
    sapdd_mg_params mp{};
    int nvec = 0, K = 0, cycles = 1;
    MgColouring cl{};
    float *P = nullptr;    // nvec FP32 fields
    float2 *Dc = nullptr;  // coarse operator, Nd * 9 * K * K
    sapdd_batch *batch = nullptr;  // kept by sapdd_mg_solve
    std::vector<void *> allocs;
};

namespace {

// Workspace of one multigrid application for `cap` systems (indexed by rhs).
struct MgWork {
    int cap = 0, nwa = 0, nwc = 0, pstride = 0;
    double *t1 = nullptr, *t2 = nullptr;  // FP64 fields: interpolated coarse solution, residual
    float2 *cb = nullptr;                 // coarse Krylov bases
    float2 *rc = nullptr, *xc = nullptr;  // coarse right-hand sides and solutions
    double *pn = nullptr, *pd = nullptr, *H = nullptr, *sc = nullptr, *beta = nullptr, *coef = nullptr;
};

template <class Alloc>
int mg_work_init(const sapdd_mg *mg, int cap, Alloc alloc, MgWork *w) {
    const Geom &g = mg->f->geo;
    const size_t nc = (size_t)g.Nd * mg->K;
    w->cap = cap;
    mg_coarse_tiling(g, mg->K, &w->nwa, &w->nwc);
    w->pstride = std::max(w->nwa, w->nwc);
    void *q;
    CHK(alloc("mg_t1", (size_t)cap * g.V * 24 * 8, &q));
    w->t1 = (double *)q;
    CHK(alloc("mg_t2", (size_t)cap * g.V * 24 * 8, &q));
    w->t2 = (double *)q;
    CHK(alloc("mg_cb", (size_t)cap * MG_BASIS_SLOTS * nc * sizeof(float2), &q));
    w->cb = (float2 *)q;
    CHK(alloc("mg_rc", (size_t)cap * nc * sizeof(float2), &q));
    w->rc = (float2 *)q;
    CHK(alloc("mg_xc", (size_t)cap * nc * sizeof(float2), &q));
    w->xc = (float2 *)q;
    CHK(alloc("mg_pn", (size_t)cap * (MG_IMAX + 1) * w->pstride * 8, &q));
    w->pn = (double *)q;
    CHK(alloc("mg_pd", (size_t)cap * 4 * MG_IMAX * w->pstride * 8, &q));
    w->pd = (double *)q;
    CHK(alloc("mg_H", (size_t)cap * (MG_IMAX + 1) * MG_IMAX * 16, &q));
    w->H = (double *)q;
    CHK(alloc("mg_sc", (size_t)cap * (MG_IMAX + 1) * 8, &q));
    w->sc = (double *)q;
    CHK(alloc("mg_beta", (size_t)cap * 8, &q));
    w->beta = (double *)q;
    CHK(alloc("mg_coef", (size_t)cap * MG_IMAX * 16, &q));
    w->coef = (double *)q;
    return SAPDD_OK;
}

MgGmres mg_gmres(const sapdd_mg *mg, const MgWork &w, const int *active) {
    const Geom &g = mg->f->geo;
    MgGmres G{};
    G.Dc = mg->Dc;
    G.K = mg->K;
    for (int mu = 0; mu < 4; ++mu) G.grid[mu] = g.G[mu];
    G.Nd = g.Nd;
    G.nwa = w.nwa;
    G.nwc = w.nwc;
    G.pstride = w.pstride;
    G.basis = w.cb;
    G.vstride = g.Nd * mg->K;
    G.bstride = MG_BASIS_SLOTS * G.vstride;
    G.fused = mg->mp.coarse_form;
    G.rc = w.rc;
    G.xc = w.xc;
    G.pn = w.pn;
    G.pd = w.pd;
    G.H = w.H;
    G.sc = w.sc;
    G.beta = w.beta;
    G.coef = w.coef;
    // one classical Gram-Schmidt pass per coarse step: a second pass left the outer step
    // count unchanged on 16^3 x 32 (229 / 230 steps) and cost a quarter of the coarse time
    G.active = active;
    return G;
}

// psi = B(s eta) for the listed systems (s = eta_scale[rhs * eta_sstride], 1 if null):
// e = P GMRES(D_c, P^H eta) (restarted GMRES(k), a homogeneous map, so it runs on the
// unscaled eta), t2 = eta - M e, psi = SAP(s t2) + s e. eta: FP64 fields with stride
// eta_stride fields per rhs; psi in psi_prec with stride psi_stride fields; per-rhs kappa
// and clover from ss.
int mg_run(sapdd_ctx *c, const sapdd_mg *mg, const MgWork &w, const SapState &ss, const sapdd_params *p,
           const double *eta, int eta_stride, const double *eta_scale, int eta_sstride, void *psi, int psi_prec,
           int psi_stride, const int *active, int nact) {
    const Geom &g = mg->f->geo;
    const int64_t NS = g.V * 24;
    const MgGmres G = mg_gmres(mg, w, active);
    const int k = mg->mp.coarse_iters;
    KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_restrict(g, mg->nvec, eta, eta_stride * NS, mg->P, w.rc, G.vstride, active,
                                                   nact, c->stream));
    KLAUNCH(c, SAPDD_K_MG_COARSE, launch_mg_coarse_gmres(G, nact, k, mg->cycles, c->stream));
    KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_prolong_basis(g, mg->nvec, mg->P, w.xc, G.vstride, 0, nullptr, 0, 1, w.t1,
                                                        NS, active, nact, c->stream));
    DslashIO io{};
    io.in = Fld{w.t1, nullptr, P64};
    io.out = Fld{w.t2, nullptr, P64};
    io.sub = eta;
    io.active = active;
    io.nact = nact;
    io.in_stride = io.out_stride = 1;
    io.sub_stride = eta_stride;
    io.kappa = ss.kappa;
    KLAUNCH(c, SAPDD_K_DSLASH, launch_dslash_full(g, links_of(mg->f, P64), tclov_of(mg->f, P64), 0.0, io, c->stream));
    CHK(sap_run(c, g, ss, p, w.t2, 1, eta_scale, eta_sstride, psi, psi_prec, psi_stride, active, nact));
    KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_axpy(g, Fld{psi, nullptr, psi_prec}, psi_stride * NS, w.t1, NS, 1.0,
                                               eta_scale, eta_sstride, active, nact, c->stream));
    return SAPDD_OK;
}

}  // namespace

// ====================================================================== FGMRES batch
// A batch holds up to `cap` right-hand sides (slots) on one field, each with its own
// kappa and Krylov state. One step is one FGMRES(m) restart cycle for every active slot:
// the SAP preconditioner, the FP64 operator and the Gram-Schmidt passes of the whole
// batch run as single launches over the active slots, and the true FP64 residual at the
// end of the cycle both decides convergence (the reliable update) and starts the next
// cycle. Slots join (sapdd_batch_add) and leave (sapdd_batch_take) between steps, which
// is what the serving loop's continuous batching uses. Every per-slot result is
// independent of which other slots share the batch: kernels treat slots independently
// and all reductions run in a fixed order.
namespace {

typedef std::complex<double> cd;

struct Slot {
    // pending: added, its |b| not read back yet (the next step does that for every
    // pending slot at once, so adding a right-hand side waits for nothing)
    bool used = false, finished = false, ready = false, dirty = false, in_cycle = false, pending = false;
    bool has_x0 = false;
    double kappa = 0, bnorm = 0, beta = 0, est = 0, true_relres = 0;
    int iters = 0, restarts = 0, converged = 0, nz = 0, status = SAPDD_OK, gap_restarts = 0;
    std::vector<cd> H, cs, sn, gv;  // Hessenberg matrix as the Givens rotations leave it
    // Deflated restarts: Hr is the cycle's Hbar as built ((m+1) x m, column-major), c0 the
    // coordinates of the residual in the basis at the cycle start, j0 the first Arnoldi
    // step of the cycle, y the last least-squares solution; `deflated` marks a cycle that
    // continues a deflated basis (dense leading block, solved without the Givens update).
    std::vector<cd> Hr, c0, y;
    int j0 = 0;
    bool deflated = false;
};

enum { SEG_CHECK = 0, SEG_CHECK2 = 1, SEG_CYCLE = 2, SEG_DEFL = 3, SEG_GROUP = 4, SEG_ADD = 5, NSEG = 10 };

}  // namespace

struct sapdd_batch {
    sapdd_ctx *c = nullptr;
    sapdd_field *f = nullptr;
    unsigned long long f_id = 0;  // the field's id at creation
    sapdd_params p{};
    int cap = 0, m = 0, k = 0, prec = 0, zprec = 0;
    Geom g{};
    int64_t NS = 0, ncx = 0;
    Fld Vb{}, Zb{}, Bb{}, Xb{};
    SapState ss{};
    double *coef = nullptr, *vscale = nullptr, *part = nullptr, *ydev = nullptr;
    double *pdev = nullptr, *hp = nullptr;  // deflation bases per slot, (m+1) x (k+1) complex (device, pinned host)
    int *dlists = nullptr;
    char *pin = nullptr;
    int *hlists = nullptr;
    double *hcoef = nullptr, *hy = nullptr;
    char *hmeta = nullptr;
    int CST = 0, hoff = 0, coff = 0, noff = 0, nwg_d = 0;
    bool use_graph = false;
    std::vector<Slot> slots;
    std::vector<void *> allocs;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    double t_sap = 0, t_d = 0, t_gs = 0, t_host = 0;
    sapdd_mg *mg = nullptr;  // multigrid preconditioner in place of SAP (sapdd_batch_set_mg)
    MgWork mw{};
    // Elastic batches (SAPDD_ELASTIC): every per-slot field is one address range of
    // cap slot ranges, each reserved on its own (the runtime takes a second mapping inside
    // one reservation badly) and backed by physical memory only while the slot is in use.
    struct Piece {  // one reservation, backed by one physical chunk while committed
        void *va = nullptr;
        size_t len = 0;
        hipMemGenericAllocationHandle_t h{};
        bool full = false;  // a full-size piece (its chunk is pooled on release)
    };
    struct EField {
        size_t data_per_slot = 0, scale_per_slot = 0;  // bytes; the scales follow all data
        int npiece = 0;                                 // pieces per slot: data, then scales
        std::vector<Piece> pieces;                      // [slot * npiece + k]
        std::vector<char> committed;
    };
    bool elastic = false;
    size_t gran = 0, fixed_bytes = 0;
    std::vector<EField> efields;
};

static const sapdd_field *batch_field(const sapdd_batch *B) { return B->f; }

namespace {

int balloc(sapdd_batch *B, size_t bytes, void **out) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(B->c, SAPDD_ENOMEM, "hipMalloc of %zu bytes for a solver batch failed", bytes);
    }
    B->allocs.push_back(q);
    B->fixed_bytes += bytes ? bytes : 16;
    *out = q;
    return SAPDD_OK;
}

hipMemAllocationProp vmm_prop(int device) {
    hipMemAllocationProp prop{};
    prop.type = hipMemAllocationTypePinned;
    prop.location.type = hipMemLocationTypeDevice;
    prop.location.id = device;
    return prop;
}

// Physical memory of the elastic batches of the process, per device: a slot's full-size
// pieces take their chunks from here when committed and give them back when trimmed, so
// memory moves between batches without being freed and allocated again (an allocation
// right after a large free waited up to 2 s on the device, which clears freed memory
// first). The pool frees its chunks when the device's last elastic batch is destroyed.
struct PhysPool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<hipMemGenericAllocationHandle_t>> free;
    std::map<int, int> batches;  // live elastic batches per device
};
PhysPool &phys_pool() {
    static PhysPool p;
    return p;
}

void pool_add_batch(int device) {
    PhysPool &pp = phys_pool();
    std::lock_guard<std::mutex> g(pp.mu);
    pp.batches[device] += 1;
}

void pool_drop_batch(int device) {
    PhysPool &pp = phys_pool();
    std::lock_guard<std::mutex> g(pp.mu);
    if (--pp.batches[device] > 0) return;
    for (auto it = pp.free.begin(); it != pp.free.end();) {
        if (it->first.first != device) {
            ++it;
            continue;
        }
        for (auto h : it->second) (void)hipMemRelease(h);
        it = pp.free.erase(it);
    }
}

// Pieces of at most 64 MiB: full pieces are interchangeable between batches of any
// lattice, only the last piece of a field has a size of its own. SAPDD_ELASTIC_PIECE_KB
// in the environment sets another size (tests use small pieces so that small lattices
// span many).
size_t piece_bytes() {
    static const size_t v = [] {
        const char *e = getenv("SAPDD_ELASTIC_PIECE_KB");
        const long long kb = e ? atoll(e) : 0;
        return kb > 0 ? (size_t)kb << 10 : (size_t)64 << 20;
    }();
    return v;
}

size_t full_piece(size_t gran) { return std::max(gran, piece_bytes() / gran * gran); }

void split_pieces(size_t len, size_t gran, std::vector<size_t> &out) {
    const size_t piece = full_piece(gran);
    for (; len > piece; len -= piece) out.push_back(piece);
    if (len) out.push_back(len);
}

// A per-slot field of nf = cap * per-slot copies: device memory (fixed batch), or in an
// elastic batch an address range whose slots are committed on admission (commit_slot).
int bfield(sapdd_batch *B, int nf, int prec, int ncomp, Fld *f) {
    const size_t nd = (size_t)B->g.V * ncomp * nf;
    size_t bytes = nd * prec_bytes(prec);
    const size_t sc_off = (bytes + 255) / 256 * 256;
    if (prec == P16) bytes = sc_off + (size_t)B->g.V * nf * sizeof(float);
    if (!B->elastic) {
        void *q;
        CHK(balloc(B, bytes, &q));
        *f = Fld{q, prec == P16 ? (float *)((char *)q + sc_off) : nullptr, prec};
        return SAPDD_OK;
    }
    const int per = nf / B->cap;
    sapdd_batch::EField e;
    e.data_per_slot = (size_t)B->g.V * ncomp * per * prec_bytes(prec);
    e.scale_per_slot = prec == P16 ? (size_t)B->g.V * per * sizeof(float) : 0;
    if (e.data_per_slot % B->gran || e.scale_per_slot % B->gran)
        return fail(B->c, SAPDD_EINVAL,
                    "an elastic batch needs per-slot fields in whole pages of %zu bytes (lattice volume a "
                    "multiple of %zu sites)", B->gran, B->gran / 4);
    std::vector<size_t> dl, sl;
    split_pieces(e.data_per_slot, B->gran, dl);
    split_pieces(e.scale_per_slot, B->gran, sl);
    e.npiece = (int)(dl.size() + sl.size());
    const size_t total = (size_t)B->cap * (e.data_per_slot + e.scale_per_slot);
    // find a free range for the whole field, then hold it as adjacent reservations, one
    // per piece (one mapping per reservation: a second mapping inside one reservation
    // made hipMemSetAccess fail on this runtime)
    void *big = nullptr;
    hipError_t err = hipMemAddressReserve(&big, total, B->gran, nullptr, 0);
    if (err == hipSuccess) err = hipMemAddressFree(big, total);
    for (int r = 0; err == hipSuccess && r < B->cap; ++r) {
        for (int part = 0; part < 2 && err == hipSuccess; ++part) {
            char *want = (char *)big + (part == 0 ? r * e.data_per_slot
                                                  : B->cap * e.data_per_slot + r * e.scale_per_slot);
            for (size_t len : part == 0 ? dl : sl) {
                void *got = nullptr;
                err = hipMemAddressReserve(&got, len, B->gran, want, 0);
                if (err != hipSuccess) break;
                e.pieces.push_back({got, len, {}, len == full_piece(B->gran)});
                if (got != want) {  // the hole was taken meanwhile
                    err = hipErrorOutOfMemory;
                    break;
                }
                want += len;
            }
        }
    }
    if (err != hipSuccess) {
        (void)hipGetLastError();
        for (auto &q : e.pieces) (void)hipMemAddressFree(q.va, q.len);
        return fail(B->c, SAPDD_ENOMEM, "reserving %zu bytes of adjacent address space failed: %s", total,
                    hipGetErrorString(err));
    }
    e.committed.assign(B->cap, 0);
    B->efields.push_back(std::move(e));
    *f = Fld{big, prec == P16 ? (float *)((char *)big + B->cap * B->efields.back().data_per_slot) : nullptr, prec};
    return SAPDD_OK;
}

// Back one piece with a chunk (from the pool, else new) readable and writable by the
// device.
hipError_t piece_commit(sapdd_batch::Piece &q, int device, const char **what) {
    const hipMemAllocationProp prop = vmm_prop(device);
    hipMemAccessDesc acc{};
    acc.location = prop.location;
    acc.flags = hipMemAccessFlagsProtReadWrite;
    bool pooled = false;
    {
        PhysPool &pp = phys_pool();
        std::lock_guard<std::mutex> g(pp.mu);
        auto it = pp.free.find({device, q.len});
        if (it != pp.free.end() && !it->second.empty()) {
            q.h = it->second.back();
            it->second.pop_back();
            pooled = true;
        }
    }
    hipError_t e = hipSuccess;
    if (!pooled) {
        *what = "hipMemCreate";
        e = hipMemCreate(&q.h, q.len, &prop, 0);
        if (e != hipSuccess) return e;
    }
    *what = "hipMemMap";
    e = hipMemMap(q.va, q.len, 0, q.h, 0);
    if (e == hipSuccess) {
        *what = "hipMemSetAccess";
        e = hipMemSetAccess(q.va, q.len, &acc, 1);
        if (e != hipSuccess) (void)hipMemUnmap(q.va, q.len);
    }
    if (e != hipSuccess) (void)hipMemRelease(q.h);
    return e;
}

// Unmap one piece (the stream must be done with it). A full-size chunk goes to the pool,
// where any elastic batch's next commit finds it before allocating anew, so the memory
// held by mapped slots and the pool together never exceeds the most the slots had mapped
// at once. The last piece of a field has a size of its own, fits no other batch's
// pieces, and is freed (at most 64 MiB, quick to clear).
void piece_release(sapdd_batch::Piece &q, int device) {
    (void)hipMemUnmap(q.va, q.len);
    if (!q.full) {
        (void)hipMemRelease(q.h);
        return;
    }
    PhysPool &pp = phys_pool();
    std::lock_guard<std::mutex> g(pp.mu);
    pp.free[{device, q.len}].push_back(q.h);
}

void vmm_release(sapdd_batch::EField &e, int r, int device) {
    if (!e.committed[r]) return;
    for (int k = 0; k < e.npiece; ++k) piece_release(e.pieces[(size_t)r * e.npiece + k], device);
    e.committed[r] = 0;
}

bool slot_committed(const sapdd_batch *B, int r) {
    return B->elastic && !B->efields.empty() && B->efields.front().committed[r];
}

// Commit slot r's memory in every elastic field; on failure nothing stays committed.
// A slot that still holds its memory from an earlier use keeps it.
int commit_slot(sapdd_batch *B, int r) {
    if (!B->elastic || slot_committed(B, r)) return SAPDD_OK;
    const int dev = B->c->device;
    const char *what = "";
    hipError_t err = hipSuccess;
    size_t i = 0;
    for (; i < B->efields.size(); ++i) {
        sapdd_batch::EField &e = B->efields[i];
        int k = 0;
        for (; k < e.npiece; ++k)
            if ((err = piece_commit(e.pieces[(size_t)r * e.npiece + k], dev, &what)) != hipSuccess) break;
        if (err != hipSuccess) {
            for (int q = 0; q < k; ++q) piece_release(e.pieces[(size_t)r * e.npiece + q], dev);
            break;
        }
        e.committed[r] = 1;
    }
    if (err == hipSuccess) return SAPDD_OK;
    (void)hipGetLastError();
    for (size_t k = 0; k < i; ++k) vmm_release(B->efields[k], r, dev);
    return fail(B->c, err == hipErrorOutOfMemory ? SAPDD_ENOMEM : SAPDD_EDEVICE,
                "committing the memory of slot %d failed: %s (%s)", r, hipGetErrorString(err), what);
}

// Release slot r's memory in every elastic field to the pool (the stream must be done
// with it).
void release_slot(sapdd_batch *B, int r) {
    if (!B->elastic) return;
    for (auto &e : B->efields) vmm_release(e, r, B->c->device);
}

int upload(sapdd_batch *B, int seg, const std::vector<int> &v, int **out) {
    int *h = B->hlists + (size_t)seg * B->cap;
    for (size_t i = 0; i < v.size(); ++i) h[i] = v[i];
    int *d = B->dlists + (size_t)seg * B->cap;
    HIPCHK(B->c, hipMemcpyAsync(d, h, v.size() * sizeof(int), hipMemcpyHostToDevice, B->c->stream));
    *out = d;
    return SAPDD_OK;
}

// Copy the coefficient blocks to the host and wait (the once-per-step sync point).
int fetch_coef(sapdd_batch *B) {
    sapdd_ctx *c = B->c;
    HIPCHK(c, hipMemcpyAsync(B->hcoef, B->coef, (size_t)B->cap * B->CST * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->prof) CHK(prof_drain(c));
    return SAPDD_OK;
}

// True residual r = b - M x of the listed slots into basis slot 0, |r|, vscale[0] = 1/|r|;
// decides convergence (tol), failure (non-finite) and exhaustion (max_iter). gap_check:
// compare with the implicit residual of the cycle that just ended (off for the second
// pass over slots the gap rule sent back to a plain restart).
int batch_residual(sapdd_batch *B, const std::vector<int> &list, bool gap_check = true) {
    if (list.empty()) return SAPDD_OK;
    sapdd_ctx *c = B->c;
    // Slots that continue a deflated basis keep basis vectors 0..k: their true residual
    // goes to the spare vector m and only its norm is used.
    std::vector<int> plain, defl;
    for (int r : list) (B->slots[r].deflated ? defl : plain).push_back(r);
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    for (int g = 0; g < 2; ++g) {
        const std::vector<int> &l = g == 0 ? plain : defl;
        if (l.empty()) continue;
        int *d_list;
        CHK(upload(B, g == 0 ? SEG_CHECK : SEG_CHECK2, l, &d_list));
        DslashIO io{};
        io.in = B->Xb;
        io.out = Fld{(double *)B->Vb.data + (g == 0 ? 0 : (size_t)B->m * B->NS), nullptr, P64};
        io.sub = (const double *)B->Bb.data;
        io.part = B->part;
        io.active = d_list;
        io.nact = (int)l.size();
        io.in_stride = 1;
        io.out_stride = B->m + 1;
        io.sub_stride = 1;
        io.kappa = B->ss.kappa;
        KLAUNCH(c, SAPDD_K_DSLASH,
                launch_dslash_full(B->g, links_of(B->f, P64), tclov_of(B->f, P64), 0.0, io, c->stream));
        KLAUNCH(c, SAPDD_K_DSLASH, launch_reduce(B->part, B->nwg_d, 1, d_list, io.nact, B->coef + B->noff, B->CST,
                                                 nullptr, 0, 0, g == 0 ? B->vscale : nullptr, B->m + 1, c->stream));
    }
    HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
    CHK(fetch_coef(B));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    B->t_d += ms * 1e-3;
    // reliable update: the implicit residual of the cycle that just ended is the
    // least-squares residual (its norm est * |b|), or for a slot continuing a deflated
    // basis the recursive residual V c0 (norm |c0|, V orthonormal)
    const double gap = B->p.gap > 0 ? B->p.gap : 10.0;
    std::vector<int> redo;
    for (int r : list) {
        Slot &s = B->slots[r];
        s.dirty = false;
        s.beta = std::sqrt(B->hcoef[(size_t)r * B->CST + B->noff]);
        s.true_relres = s.beta / s.bnorm;
        s.ready = false;
        double implicit = -1;
        if (!gap_check) {
        } else if (s.deflated) {
            double q = 0;
            for (const cd &v : s.c0) q += std::norm(v);
            implicit = std::sqrt(q);
        } else if (s.restarts > 0) {
            implicit = s.est * s.bnorm;
        }
        if (implicit >= 0 && std::isfinite(s.beta) && s.beta > gap * implicit) {
            s.gap_restarts += 1;
            if (s.deflated && s.true_relres > B->p.tol && s.iters < B->p.max_iter) {
                // restart now from the true residual, computed into basis vector 0 below
                s.deflated = false;
                redo.push_back(r);
                continue;
            }
        }
        if (!std::isfinite(s.beta)) {
            s.status = SAPDD_ENAN;
            s.finished = true;
        } else if (s.true_relres <= B->p.tol) {
            s.converged = 1;
            s.finished = true;
        } else if (s.iters >= B->p.max_iter) {
            s.status = SAPDD_ENOCONV;
            s.finished = true;
        } else {
            s.ready = true;
        }
    }
    if (!redo.empty()) return batch_residual(B, redo, false);
    return SAPDD_OK;
}

// z_j = SAP(v_j), or the multigrid cycle B(v_j) when the batch has one, for the cycle
// list (device list in segment SEG_CYCLE, ncyc slots),
// replayed from a graph captured once per (ncyc, j) when graphs are enabled.
int batch_sap(sapdd_batch *B, int j, const int *d_cyc, int ncyc) {
    sapdd_ctx *c = B->c;
    const double *eta = (const double *)B->Vb.data + (size_t)j * B->NS;
    void *psi = (char *)B->Zb.data + (size_t)j * B->NS * prec_bytes(B->zprec);
    auto run = [&]() {
        if (B->mg)
            return mg_run(c, B->mg, B->mw, B->ss, &B->p, eta, B->m + 1, B->vscale + j, B->m + 1, psi, B->zprec, B->m,
                          d_cyc, ncyc);
        return sap_run(c, B->g, B->ss, &B->p, eta, B->m + 1, B->vscale + j, B->m + 1, psi, B->zprec, B->m, d_cyc,
                       ncyc);
    };
    if (!B->use_graph) return run();
    auto key = std::make_pair(ncyc, j);
    auto it = B->graphs.find(key);
    if (it == B->graphs.end()) {
        const bool prof = c->prof;
        c->prof = false;  // no event records inside the captured sequence
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int r = run();
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &graph);
        c->prof = prof;
        if (r != SAPDD_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        HIPCHK(c, e);
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(c, e);
        it = B->graphs.emplace(key, exec).first;
    }
    CHK(prof_begin(c, SAPDD_K_SAP_HALF));
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    CHK(prof_end(c, 2 * B->p.ncy));
    return SAPDD_OK;
}

// Deflated restart of slot r after a full cycle (flexible GMRES with deflated restarts,
// Sec. 3.1, in the form of Morgan's GMRES-DR): with Hbar = Hr ((m+1) x m), y the
// cycle's least-squares solution and s = c0 - Hbar y the residual's coordinates,
//   harmonic Ritz: (H_m + H_m^-H h^H h) g = theta g  (H_m = first m rows, h = last row);
//   P_k = the Schur vectors of the k values of smallest modulus (orthonormal, m x k);
//   P_{k+1} = [[P_k; 0], s orthogonalised against them and normalised];
//   next cycle: V <- V P_{k+1}, Z <- Z P_k, Hbar <- P_{k+1}^H Hbar P_k, c0 <- P_{k+1}^H s,
//   first step k. P_{k+1} goes to the slot's block of the pinned staging area (column-major,
//   leading dimension m+1). Returns false (plain restart) if H_m is singular, the Schur
//   iteration fails or s vanishes.
bool deflate_basis(sapdd_batch *B, int r) {
    Slot &s = B->slots[r];
    const int m = B->m, k = B->k, M1 = m + 1;
    if ((int)s.y.size() != m) return false;
    std::vector<cd> sres(M1);
    for (int i = 0; i < M1; ++i) {
        cd t = s.c0[i];
        for (int q = 0; q < m; ++q) t -= s.Hr[i + (size_t)M1 * q] * s.y[q];
        sres[i] = t;
    }
    std::vector<cd> hmh((size_t)m * m), f(m), a((size_t)m * m), q;
    for (int i = 0; i < m; ++i) {
        f[i] = std::conj(s.Hr[m + (size_t)M1 * i]);
        for (int j = 0; j < m; ++j) {
            hmh[i + (size_t)m * j] = std::conj(s.Hr[j + (size_t)M1 * i]);
            a[i + (size_t)m * j] = s.Hr[i + (size_t)M1 * j];
        }
    }
    if (!dense::solve(m, hmh, f)) return false;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) a[i + (size_t)m * j] += f[i] * s.Hr[m + (size_t)M1 * j];
    if (!dense::schur_sorted(m, a, q)) return false;
    std::vector<cd> P((size_t)M1 * (k + 1), 0.0);
    for (int l = 0; l < k; ++l)
        for (int i = 0; i < m; ++i) P[i + (size_t)M1 * l] = q[i + (size_t)m * l];
    std::vector<cd> v = sres;
    for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < k; ++l) {
            cd d = 0;
            for (int i = 0; i < M1; ++i) d += std::conj(P[i + (size_t)M1 * l]) * v[i];
            for (int i = 0; i < M1; ++i) v[i] -= d * P[i + (size_t)M1 * l];
        }
    double nv = 0;
    for (const cd &x : v) nv += std::norm(x);
    nv = std::sqrt(nv);
    if (!(nv > 0) || !std::isfinite(nv)) return false;
    for (int i = 0; i < M1; ++i) P[i + (size_t)M1 * k] = v[i] / nv;
    // Hbar_new = P^H Hbar P_k, c0_new = P^H s
    std::vector<cd> hp_((size_t)M1 * k);  // Hbar P_k, (m+1) x k
    for (int b = 0; b < k; ++b)
        for (int i = 0; i < M1; ++i) {
            cd t = 0;
            for (int qq = 0; qq < m; ++qq) t += s.Hr[i + (size_t)M1 * qq] * P[qq + (size_t)M1 * b];
            hp_[i + (size_t)M1 * b] = t;
        }
    std::vector<cd> hn((size_t)M1 * m, 0.0), cn(M1, 0.0);
    for (int a2 = 0; a2 <= k; ++a2) {
        for (int b = 0; b < k; ++b) {
            cd t = 0;
            for (int i = 0; i < M1; ++i) t += std::conj(P[i + (size_t)M1 * a2]) * hp_[i + (size_t)M1 * b];
            hn[a2 + (size_t)M1 * b] = t;
        }
        cd t = 0;
        for (int i = 0; i < M1; ++i) t += std::conj(P[i + (size_t)M1 * a2]) * sres[i];
        cn[a2] = t;
    }
    double *hp = B->hp + (size_t)r * M1 * (k + 1) * 2;
    for (size_t i = 0; i < P.size(); ++i) {
        hp[2 * i] = P[i].real();
        hp[2 * i + 1] = P[i].imag();
    }
    s.Hr = hn;
    s.c0 = cn;
    s.j0 = k;
    return true;
}

// One FGMRES(m) restart cycle over every ready slot. A slot that continues a deflated
// basis starts at Arnoldi step k; with deflation (k > 0) every full cycle ends with the
// deflated restart of the next (deflate_basis).
int batch_cycle(sapdd_batch *B) {
    sapdd_ctx *c = B->c;
    const int m = B->m;
    std::vector<int> running;
    for (int r = 0; r < B->cap; ++r)
        if (B->slots[r].used && !B->slots[r].finished && B->slots[r].ready) running.push_back(r);
    if (running.empty()) return SAPDD_OK;
    int jmin = m;
    for (int r : running) {
        Slot &s = B->slots[r];
        s.in_cycle = true;
        s.nz = 0;
        if (!s.deflated) {
            std::fill(s.H.begin(), s.H.end(), 0.0);
            std::fill(s.gv.begin(), s.gv.end(), 0.0);
            s.gv[0] = s.beta;
            s.Hr.assign((size_t)(m + 1) * m, 0.0);
            s.c0.assign(m + 1, 0.0);
            s.c0[0] = s.beta;
            s.j0 = 0;
        }
        jmin = std::min(jmin, s.j0);
    }
    const std::vector<int> members = running;
    std::vector<int> cycle;  // the slots of the current step, as uploaded
    int *d_cyc = nullptr;
    int ncyc = 0;
    double *Vd = (double *)B->Vb.data;
    const int nwg = blas_partials(B->ncx, 1);
    for (int j = jmin; j < m && !running.empty(); ++j) {
        std::vector<int> act;
        for (int r : running)
            if (B->slots[r].j0 <= j) act.push_back(r);
        if (act.empty()) continue;
        if (act != cycle) {
            cycle = act;
            ncyc = (int)cycle.size();
            CHK(upload(B, SEG_CYCLE, cycle, &d_cyc));
        }
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        CHK(batch_sap(B, j, d_cyc, ncyc));
        HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
        // w = M z_j into basis slot j + 1
        DslashIO w{};
        w.in = Fld{(char *)B->Zb.data + (size_t)j * B->NS * prec_bytes(B->zprec), nullptr, B->zprec};
        w.out = Fld{Vd + (size_t)(j + 1) * B->NS, nullptr, P64};
        w.active = d_cyc;
        w.nact = ncyc;
        w.in_stride = m;
        w.out_stride = m + 1;
        w.kappa = B->ss.kappa;
        KLAUNCH(c, SAPDD_K_DSLASH,
                launch_dslash_full(B->g, links_of(B->f, P64), tclov_of(B->f, P64), 0.0, w, c->stream));
        HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
        // classical Gram-Schmidt, twice: h = V^H w; w' = w - V h, c = V^H w' and |w'|^2 in
        // one pass; w'' = w' - V c and |w''|^2 in one pass, skipped for a slot whose
        // correction is negligible, |c| <= 1e-9 |w'| (w'' = w' then, and the Hessenberg
        // column takes h alone, so M z_j = V h + w'' holds as computed)
        CgsArgs a{};
        a.vbase = Vd;
        a.vstride = B->NS;
        a.rstride = (int64_t)(m + 1) * B->NS;
        a.vscale = B->vscale;
        a.vsstride = m + 1;
        a.w = Vd + (size_t)(j + 1) * B->NS;
        a.wstride = (int64_t)(m + 1) * B->NS;
        a.cstride = B->CST;
        a.part = B->part;
        a.active = d_cyc;
        a.nact = ncyc;
        a.n = B->ncx;
        a.v0 = 0;
        a.nv = j + 1;
        KLAUNCH(c, SAPDD_K_GS, launch_cgs(0, a, c->stream));
        KLAUNCH(c, SAPDD_K_GS, launch_reduce(B->part, nwg, 2 * a.nv, d_cyc, ncyc, B->coef + B->hoff, B->CST,
                                             B->vscale, m + 1, 0, nullptr, 0, c->stream));
        a.coef = B->coef + B->hoff;
        KLAUNCH(c, SAPDD_K_GS, launch_cgs(1, a, c->stream));
        KLAUNCH(c, SAPDD_K_GS, launch_reduce(B->part, nwg, 2 * a.nv + 1, d_cyc, ncyc, B->coef + B->coff, B->CST,
                                             B->vscale, m + 1, 0, nullptr, 0, c->stream));
        a.coef = B->coef + B->coff;
        a.skip_tol = CGS_SKIP_TOL;
        KLAUNCH(c, SAPDD_K_GS, launch_cgs(2, a, c->stream));
        KLAUNCH(c, SAPDD_K_GS, launch_reduce(B->part, nwg, 1, d_cyc, ncyc, B->coef + B->noff, B->CST, nullptr, 0, 0,
                                             B->vscale + j + 1, m + 1, c->stream));
        HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
        CHK(fetch_coef(B));
        const double th = now_s();
        {
            float ms;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
            B->t_sap += ms * 1e-3;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
            B->t_d += ms * 1e-3;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
            B->t_gs += ms * 1e-3;
        }
        // host: Hessenberg column, Givens rotations, least-squares residual estimate
        std::vector<int> stopped;
        for (int r : cycle) {
            Slot &s = B->slots[r];
            const double *hc = B->hcoef + (size_t)r * B->CST;
            cd *hr = &s.Hr[(size_t)(m + 1) * j];
            // the device's test, on the same numbers: was the second correction skipped?
            double cc = 0;
            for (int i = 0; i <= j; ++i)
                cc += hc[B->coff + 2 * i] * hc[B->coff + 2 * i] + hc[B->coff + 2 * i + 1] * hc[B->coff + 2 * i + 1];
            const double second = cc <= CGS_SKIP_TOL * hc[B->coff + 2 * (j + 1)] ? 0.0 : 1.0;
            for (int i = 0; i <= j; ++i)
                hr[i] = cd(hc[B->hoff + 2 * i] + second * hc[B->coff + 2 * i],
                           hc[B->hoff + 2 * i + 1] + second * hc[B->coff + 2 * i + 1]);
            const double hn = std::sqrt(std::max(0.0, hc[B->noff]));
            hr[j + 1] = hn;
            if (s.deflated) {  // dense leading block: least squares from scratch
                std::vector<cd> hsub((size_t)(j + 2) * (j + 1));
                for (int q = 0; q <= j; ++q)
                    for (int i = 0; i < j + 2; ++i) hsub[i + (size_t)(j + 2) * q] = s.Hr[i + (size_t)(m + 1) * q];
                const double res = dense::lstsq(j + 2, j + 1, hsub, std::vector<cd>(s.c0.begin(), s.c0.begin() + j + 2),
                                                s.y);
                s.est = res / s.bnorm;
                s.iters += 1;
                s.nz = j + 1;
                if (!std::isfinite(s.est)) {
                    s.status = SAPDD_ENAN;
                    s.in_cycle = false;
                    s.nz = 0;
                    stopped.push_back(r);
                } else if (s.est <= B->p.tol || hn == 0.0 || s.iters >= B->p.max_iter) {
                    s.in_cycle = false;
                    stopped.push_back(r);
                }
                continue;
            }
            cd *col = &s.H[(size_t)(m + 1) * j];
            for (int i = 0; i <= j + 1; ++i) col[i] = hr[i];
            for (int i = 0; i < j; ++i) {
                const cd t = std::conj(s.cs[i]) * col[i] + std::conj(s.sn[i]) * col[i + 1];
                col[i + 1] = -s.sn[i] * col[i] + s.cs[i] * col[i + 1];
                col[i] = t;
            }
            const double den = std::sqrt(std::norm(col[j]) + std::norm(col[j + 1]));
            cd cj = 1.0, sj = 0.0;
            if (den > 0) {
                cj = col[j] / den;
                sj = col[j + 1] / den;
            }
            s.cs[j] = cj;
            s.sn[j] = sj;
            col[j] = den;
            col[j + 1] = 0.0;
            s.gv[j + 1] = -sj * s.gv[j];
            s.gv[j] = std::conj(cj) * s.gv[j];
            s.est = std::abs(s.gv[j + 1]) / s.bnorm;
            s.iters += 1;
            s.nz = j + 1;
            if (!std::isfinite(s.est) || den == 0.0) {  // the x update below is skipped for this slot
                if (!std::isfinite(s.est)) s.status = SAPDD_ENAN;
                s.in_cycle = false;
                if (!std::isfinite(s.est)) s.nz = 0;
                stopped.push_back(r);
                continue;
            }
            if (s.est <= B->p.tol || hn == 0.0 || s.iters >= B->p.max_iter) {
                s.in_cycle = false;
                stopped.push_back(r);
                continue;
            }
        }
        B->t_host += now_s() - th;
        if (!stopped.empty()) {
            std::vector<int> keep;
            for (int r : running)
                if (std::find(stopped.begin(), stopped.end(), r) == stopped.end()) keep.push_back(r);
            running = keep;
        }
    }
    // x += Z y, one launch per basis size
    std::map<int, std::vector<int>> groups;
    for (int r : members)
        if (B->slots[r].nz > 0) groups[B->slots[r].nz].push_back(r);
    for (auto &kv : groups) {
        const int nz = kv.first;
        for (int r : kv.second) {
            Slot &s = B->slots[r];
            if (!s.deflated) {
                s.y.assign(nz, 0.0);
                for (int i = nz - 1; i >= 0; --i) {  // back substitution R y = g
                    cd t = s.gv[i];
                    for (int k = i + 1; k < nz; ++k) t -= s.H[(size_t)(m + 1) * k + i] * s.y[k];
                    const cd d = s.H[(size_t)(m + 1) * i + i];
                    s.y[i] = d != 0.0 ? t / d : 0.0;
                }
            }
            const std::vector<cd> &y = s.y;
            for (int i = 0; i < nz; ++i) {
                B->hy[(size_t)r * 2 * m + 2 * i] = y[i].real();
                B->hy[(size_t)r * 2 * m + 2 * i + 1] = y[i].imag();
            }
        }
    }
    HIPCHK(c, hipMemcpyAsync(B->ydev, B->hy, (size_t)B->cap * 2 * m * 8, hipMemcpyHostToDevice, c->stream));
    int seg = SEG_GROUP;
    for (auto &kv : groups) {
        if (seg == NSEG) {  // every staging segment in flight: let them land first
            HIPCHK(c, hipStreamSynchronize(c->stream));
            seg = SEG_GROUP;
        }
        int *d_grp;
        CHK(upload(B, seg++, kv.second, &d_grp));
        KLAUNCH(c, SAPDD_K_UPDATE, launch_zupdate((double *)B->Xb.data, B->NS, B->Zb.data, B->zprec, B->NS,
                                                  (int64_t)m * B->NS, B->ydev, 2 * m, kv.first, d_grp,
                                                  (int)kv.second.size(), B->ncx, B->g.Vbh, c->stream));
    }
    // deflated restarts: the next cycle of every slot that ran all m steps continues from
    // the recombined basis; the others restart plainly from their true residual
    if (B->k > 0) {
        std::vector<int> dr;
        for (int r : members) {
            Slot &s = B->slots[r];
            const bool full = s.nz == m && s.status == SAPDD_OK;
            s.deflated = full && deflate_basis(B, r);
            if (s.deflated) dr.push_back(r);
        }
        if (!dr.empty()) {
            const int M1 = m + 1;
            const int64_t pstride = (int64_t)M1 * (B->k + 1) * 2;
            HIPCHK(c, hipMemcpyAsync(B->pdev, B->hp, (size_t)B->cap * pstride * 8, hipMemcpyHostToDevice, c->stream));
            int *d_dr;
            CHK(upload(B, SEG_DEFL, dr, &d_dr));
            KLAUNCH(c, SAPDD_K_GS, launch_recombine(Vd, (int64_t)M1 * B->NS, B->NS, B->vscale, M1, B->pdev, pstride, M1,
                                                    M1, B->k + 1, d_dr, (int)dr.size(), B->ncx, c->stream));
            KLAUNCH(c, SAPDD_K_GS, launch_recombine((double *)B->Zb.data, (int64_t)m * B->NS, B->NS, nullptr, 0,
                                                    B->pdev, pstride, M1, m, B->k, d_dr, (int)dr.size(), B->ncx,
                                                    c->stream));
        }
    }
    std::vector<int> check;
    for (int r : members) {
        Slot &s = B->slots[r];
        s.restarts += 1;
        s.in_cycle = false;
        s.ready = false;
        if (s.status == SAPDD_ENAN) {
            s.finished = true;
            continue;
        }
        if (s.nz > 0) s.dirty = true;
        s.nz = 0;
        check.push_back(r);
    }
    return batch_residual(B, check);
}

void batch_free(sapdd_batch *B) {
    if (!B) return;
    if (B->c) (void)hipStreamSynchronize(B->c->stream);
    for (auto &kv : B->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &s : B->slots)
        if (s.used) sap_clover_release(B->f, s.kappa, lprec(B->prec));
    for (void *q : B->allocs) (void)hipFree(q);
    for (auto &e : B->efields) {
        for (int r = 0; r < (int)e.committed.size(); ++r) vmm_release(e, r, B->c->device);
        for (auto &q : e.pieces) (void)hipMemAddressFree(q.va, q.len);
    }
    if (B->elastic) pool_drop_batch(B->c->device);
    if (B->pin) (void)hipHostFree(B->pin);
    delete B;
}

// A batch kept between solve calls serves a new call with the same field, shape and
// solver parameters (tolerance and iteration cap are per call).
bool batch_reusable(const sapdd_batch *B, const sapdd_field *f, const sapdd_params *p, int nrhs) {
    return B && B->f == f && B->f_id == f->id && B->cap >= nrhs && B->p.restart == p->restart && B->p.nmr == p->nmr &&
           B->p.ncy == p->ncy && B->p.sap_prec == p->sap_prec && B->p.deflate == p->deflate &&
           ((B->p.flags ^ p->flags) & SAPDD_NO_GRAPH) == 0;
}

// Free the slots a call that failed half way may have left behind.
int batch_release_slots(sapdd_batch *B) {
    for (int r = 0; r < B->cap; ++r)
        if (B->slots[r].used) {
            sap_clover_release(B->f, B->slots[r].kappa, lprec(B->prec));
            release_slot(B, r);
            B->slots[r].used = false;
        }
    return SAPDD_OK;
}

int batch_solve_all(sapdd_batch *B, const double *kappa, const sapdd_params *p, int nrhs, const double *b, double *x,
                    sapdd_stats *stats, double t0);

}  // namespace

extern "C" {

int sapdd_batch_create(sapdd_ctx *c, const sapdd_field *fc, const sapdd_params *p, int cap, sapdd_batch **out) {
    if (!c || !fc || !out) return fail(c, SAPDD_EINVAL, "null argument");
    *out = nullptr;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_field *f = const_cast<sapdd_field *>(fc);
    CHK(check_params(c, f, p));
    // the fused correct-and-dot Gram-Schmidt pass holds all basis vectors of a step at once
    if (p->restart < 1 || p->restart > 16) return fail(c, SAPDD_EINVAL, "restart must be in 1..16");
    if (p->deflate < 0 || p->deflate >= p->restart)
        return fail(c, SAPDD_EINVAL, "deflate must be in 0..restart-1");
    if (!(p->tol > 0) || p->max_iter < 1) return fail(c, SAPDD_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (cap < 1) return fail(c, SAPDD_EINVAL, "a batch needs at least one slot");
    sapdd_batch *B = new sapdd_batch;
    B->c = c;
    B->f = f;
    B->f_id = f->id;
    B->p = *p;
    B->cap = cap;
    B->m = p->restart;
    B->prec = p->sap_prec;
    B->k = p->deflate;
    // deflated restarts recombine Z: FP64 keeps M Z = V Hbar exact through the recombination
    B->zprec = B->prec == P64 || B->k > 0 ? P64 : P32;
    B->g = f->geo;
    B->NS = B->g.V * 24;
    B->ncx = B->g.V * 12;
    B->hoff = 0;
    B->coff = 2 * (B->m + 1);
    B->noff = 4 * (B->m + 1);
    B->CST = 4 * (B->m + 1) + 2;
    B->nwg_d = dslash_full_partials(B->g);
    B->use_graph = !(p->flags & SAPDD_NO_GRAPH) && c->stream != nullptr;
    B->elastic = (p->flags & SAPDD_ELASTIC) != 0;
    if (B->elastic) {
        const hipMemAllocationProp prop = vmm_prop(c->device);
        size_t g = 0;
        const hipError_t e = hipMemGetAllocationGranularity(&g, &prop, hipMemAllocationGranularityRecommended);
        if (e != hipSuccess || g == 0) {
            (void)hipGetLastError();
            delete B;
            return fail(c, SAPDD_EDEVICE, "elastic batches need virtual memory management: %s", hipGetErrorString(e));
        }
        B->gran = g;
        pool_add_batch(c->device);  // batch_free drops it again
    }
    B->slots.resize(cap);
    for (auto &s : B->slots) {
        s.H.assign((size_t)(B->m + 1) * B->m, 0.0);
        s.cs.assign(B->m, 0.0);
        s.sn.assign(B->m, 0.0);
        s.gv.assign(B->m + 1, 0.0);
    }
    int r = SAPDD_OK;
    void *q = nullptr;
    const int nwg_b = blas_partials(B->ncx, 1);
    const size_t meta_bytes = (size_t)cap * (2 * sizeof(void *) + sizeof(double));
    do {
        if ((r = lo_copies(c, f, lprec(B->prec))) != SAPDD_OK) break;
        if (B->elastic && (r = reserve_clover_cache(c, f, lprec(B->prec))) != SAPDD_OK) break;
        if ((r = bfield(B, cap * (B->m + 1), P64, 24, &B->Vb)) != SAPDD_OK) break;
        if ((r = bfield(B, cap * B->m, B->zprec, 24, &B->Zb)) != SAPDD_OK) break;
        if ((r = bfield(B, cap, P64, 24, &B->Bb)) != SAPDD_OK) break;
        if ((r = bfield(B, cap, P64, 24, &B->Xb)) != SAPDD_OK) break;
        if ((r = bfield(B, cap, sprec(B->prec), 12, &B->ss.rres)) != SAPDD_OK) break;
        if ((r = bfield(B, cap, sprec(B->prec), 24, &B->ss.delta)) != SAPDD_OK) break;
        if ((r = balloc(B, meta_bytes, &q)) != SAPDD_OK) break;
        B->ss.X = (const void **)q;
        B->ss.Xsc = (const float **)((char *)q + cap * sizeof(void *));
        B->ss.kappa = (double *)((char *)q + 2 * cap * sizeof(void *));
        B->ss.links = links_of(f, lprec(B->prec));
        if ((r = balloc(B, (size_t)cap * B->CST * 8, &q)) != SAPDD_OK) break;
        B->coef = (double *)q;
        if ((r = balloc(B, (size_t)cap * (B->m + 1) * 8, &q)) != SAPDD_OK) break;
        B->vscale = (double *)q;
        // Gram-Schmidt partials: up to 2 * 16 + 1 values per workgroup and slot
        if ((r = balloc(B, (size_t)cap * std::max(B->nwg_d, nwg_b * 33) * 8, &q)) != SAPDD_OK) break;
        B->part = (double *)q;
        if ((r = balloc(B, (size_t)cap * 2 * B->m * 8, &q)) != SAPDD_OK) break;
        B->ydev = (double *)q;
        if ((r = balloc(B, (size_t)NSEG * cap * sizeof(int), &q)) != SAPDD_OK) break;
        B->dlists = (int *)q;
        const size_t pbytes = (size_t)cap * (B->m + 1) * (B->k + 1) * 16;
        if ((r = balloc(B, pbytes, &q)) != SAPDD_OK) break;
        B->pdev = (double *)q;
        const size_t pin_bytes = (size_t)NSEG * cap * sizeof(int) + (size_t)cap * B->CST * 8 +
                                 (size_t)cap * 2 * B->m * 8 + meta_bytes + pbytes;
        if (hipHostMalloc((void **)&B->pin, pin_bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            r = fail(c, SAPDD_ENOMEM, "pinned staging allocation failed");
            break;
        }
        B->hlists = (int *)B->pin;
        B->hcoef = (double *)(B->pin + (size_t)NSEG * cap * sizeof(int));
        B->hy = B->hcoef + (size_t)cap * B->CST;
        B->hmeta = (char *)(B->hy + (size_t)cap * 2 * B->m);
        B->hp = (double *)(B->hmeta + meta_bytes);
        memset(B->hy, 0, (size_t)cap * 2 * B->m * 8);
    } while (false);
    if (r != SAPDD_OK) {
        batch_free(B);
        return r;
    }
    *out = B;
    return SAPDD_OK;
}

int sapdd_batch_destroy(sapdd_batch *B) {
    batch_free(B);
    return SAPDD_OK;
}

long long sapdd_batch_memory(const sapdd_batch *B, long long *slot_bytes) {
    if (!B) return -1;
    long long held = (long long)B->fixed_bytes, slot = 0;
    for (const auto &e : B->efields) {
        const long long per = (long long)(e.data_per_slot + e.scale_per_slot);
        for (char c : e.committed) held += c ? per : 0;
        slot += per;
    }
    if (slot_bytes) *slot_bytes = slot;
    return held;
}

long long sapdd_batch_trim(sapdd_batch *B, int keep) {
    if (!B || keep < 0) return -1;
    sapdd_ctx *c = B->c;
    c->err.clear();
    if (!B->elastic) return 0;
    if (hipSetDevice(c->device) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, SAPDD_EDEVICE, "synchronising the batch's stream failed");
    }
    long long per = 0;
    for (const auto &e : B->efields) per += (long long)(e.data_per_slot + e.scale_per_slot);
    int warm = 0;
    long long freed = 0;
    for (int r = 0; r < B->cap; ++r) {
        if (B->slots[r].used || !slot_committed(B, r)) continue;
        if (warm < keep) {
            ++warm;
            continue;
        }
        release_slot(B, r);
        freed += per;
    }
    return freed;
}

int sapdd_batch_add(sapdd_batch *B, double kappa, const double *b, const double *x0, int flags, int *slot_out) {
    if (!B || !b || !slot_out) return SAPDD_EINVAL;
    sapdd_ctx *c = B->c;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    if (!(kappa > 0)) return fail(c, SAPDD_EINVAL, "kappa must be > 0");
    if (B->mg && kappa != B->mg->kappa)
        return fail(c, SAPDD_EINVAL, "the batch's multigrid preconditioner was built for kappa = %.17g", B->mg->kappa);
    // a free slot whose memory an elastic batch still holds first, else the first free one
    int r = -1;
    for (int q = 0; q < B->cap; ++q)
        if (!B->slots[q].used && (r < 0 || slot_committed(B, q))) {
            r = q;
            if (!B->elastic || slot_committed(B, q)) break;
        }
    if (r < 0) return fail(c, SAPDD_EFULL, "no free slot in the batch (capacity %d)", B->cap);
    Fld xf;
    CHK(sap_clover(c, B->f, kappa, lprec(B->prec), &xf, true));
    if (int rc = commit_slot(B, r); rc != SAPDD_OK) {
        sap_clover_release(B->f, kappa, lprec(B->prec));
        return rc;
    }
    Slot &s = B->slots[r];
    s = Slot();
    s.H.assign((size_t)(B->m + 1) * B->m, 0.0);
    s.cs.assign(B->m, 0.0);
    s.sn.assign(B->m, 0.0);
    s.gv.assign(B->m + 1, 0.0);
    s.used = true;
    s.kappa = kappa;
    // per-slot clover pointers and kappa for the kernels
    hipLaunchKernelGGL(slot_meta_kernel, dim3(1), dim3(1), 0, c->stream, (const void **)B->ss.X,
                       (const float **)B->ss.Xsc, B->ss.kappa, r, (const void *)xf.data, (const float *)xf.scale,
                       kappa);
    HIPCHK(c, hipGetLastError());
    // b and x into the device layout
    const double *src;
    CHK(stage_in(c, "stage_in", b, (size_t)B->NS, flags, &src));
    Fld bslot{(double *)B->Bb.data + (size_t)r * B->NS, nullptr, P64};
    HIPCHK(c, launch_pack(B->g, 24, 1, src, bslot, c->stream));
    double *xslot = (double *)B->Xb.data + (size_t)r * B->NS;
    if (x0) {
        CHK(stage_in(c, "stage_in2", x0, (size_t)B->NS, flags, &src));
        HIPCHK(c, launch_pack(B->g, 24, 1, src, Fld{xslot, nullptr, P64}, c->stream));
    } else {
        HIPCHK(c, launch_zero(xslot, B->NS, c->stream));
    }
    // |b|. From x0 = 0 the first residual is b itself: it goes straight into basis slot 0
    // with vscale[0] = 1/|b|, and no operator application is needed for it.
    double *v0slot = (double *)B->Vb.data + (size_t)r * (B->m + 1) * B->NS;
    if (!x0) HIPCHK(c, launch_copy(bslot.data, v0slot, (int64_t)B->NS * 8, c->stream));
    // |b|^2 into the slot's coefficient row (and 1/|b| into vscale[0] from a zero start):
    // the slot list comes from a kernel argument too, one int of the slot's own row of
    // the list area, so nothing here needs the stream to be idle
    int *d_one = B->dlists + (size_t)SEG_ADD * B->cap + r;
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, c->stream, d_one, r);
    HIPCHK(c, hipGetLastError());
    CgsArgs a{};
    a.w = (double *)B->Bb.data;
    a.wstride = B->NS;
    a.part = B->part;  // stream order separates it from the next add's use
    a.active = d_one;
    a.nact = 1;
    a.nv = 0;
    a.n = B->ncx;
    KLAUNCH(c, SAPDD_K_GS, launch_cgs(2, a, c->stream));
    KLAUNCH(c, SAPDD_K_GS, launch_reduce(B->part, blas_partials(B->ncx, 1), 1, d_one, 1, B->coef + B->noff, B->CST,
                                         nullptr, 0, 0, x0 ? nullptr : B->vscale, B->m + 1, c->stream));
    s.pending = true;
    s.has_x0 = x0 != nullptr;
    // host arrays may be pinned, and a pinned source is read by the copy after this
    // call returns: wait for it, so the caller may reuse b and x0 at once
    if (!(flags & SAPDD_DEVICE_PTRS)) HIPCHK(c, hipStreamSynchronize(c->stream));
    *slot_out = r;
    return SAPDD_OK;
}

}  // extern "C"

namespace {
// Read back |b| of every slot added since the last step (one wait for all of them) and
// set each one's state: finished (b = 0 or not finite), first residual due (x0 given), or
// ready for its first cycle.
int resolve_pending(sapdd_batch *B) {
    bool any = false;
    for (auto &s : B->slots) any |= s.used && s.pending;
    if (!any) return SAPDD_OK;
    sapdd_ctx *c = B->c;
    CHK(fetch_coef(B));
    for (int r = 0; r < B->cap; ++r) {
        Slot &s = B->slots[r];
        if (!s.used || !s.pending) continue;
        s.pending = false;
        double *xslot = (double *)B->Xb.data + (size_t)r * B->NS;
        s.bnorm = std::sqrt(B->hcoef[(size_t)r * B->CST + B->noff]);
        if (s.bnorm == 0.0) {
            HIPCHK(c, launch_zero(xslot, B->NS, c->stream));
            s.finished = true;
            s.converged = 1;
        } else if (!std::isfinite(s.bnorm)) {
            s.finished = true;
            s.status = SAPDD_ENAN;
        } else if (s.has_x0) {
            s.dirty = true;  // its first residual b - M x0 is computed by this step
        } else {
            s.beta = s.bnorm;  // the residual bookkeeping of batch_residual for r = b
            s.true_relres = 1.0;
            if (s.true_relres <= B->p.tol) {
                s.converged = 1;
                s.finished = true;
            } else if (s.iters >= B->p.max_iter) {
                s.status = SAPDD_ENOCONV;
                s.finished = true;
            } else {
                s.ready = true;
            }
        }
    }
    return SAPDD_OK;
}
}  // namespace

extern "C" {

int sapdd_batch_step(sapdd_batch *B, int *n_running) {
    if (!B) return SAPDD_EINVAL;
    sapdd_ctx *c = B->c;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    CHK(resolve_pending(B));
    std::vector<int> check;
    for (int r = 0; r < B->cap; ++r)
        if (B->slots[r].used && !B->slots[r].finished && B->slots[r].dirty) check.push_back(r);
    CHK(batch_residual(B, check));
    CHK(batch_cycle(B));
    int n = 0;
    for (auto &s : B->slots) n += s.used && !s.finished;
    if (n_running) *n_running = n;
    return SAPDD_OK;
}

int sapdd_batch_poll(const sapdd_batch *B, int slot, sapdd_stats *st) {
    if (!B || slot < 0 || slot >= B->cap || !B->slots[slot].used) return SAPDD_EINVAL;
    const Slot &s = B->slots[slot];
    if (st) {
        st->iters = s.iters;
        st->restarts = s.restarts;
        st->converged = s.converged;
        st->true_relres = s.true_relres;
        st->implicit_relres = s.est;
        st->t_total = 0;
        st->t_sap = B->t_sap;
        st->t_dslash = B->t_d;
        st->t_gs = B->t_gs;
        st->t_host = B->t_host;
        st->gap_restarts = s.gap_restarts;
    }
    return s.finished ? 1 : 0;
}

int sapdd_batch_take(sapdd_batch *B, int slot, double *x, int flags, sapdd_stats *st) {
    if (!B || !x || slot < 0 || slot >= B->cap || !B->slots[slot].used) return SAPDD_EINVAL;
    sapdd_ctx *c = B->c;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    Slot &s = B->slots[slot];
    sapdd_batch_poll(B, slot, st);
    double *dst = x;
    if (!(flags & SAPDD_DEVICE_PTRS)) {
        void *d;
        CHK(buf(c, "stage_out", (size_t)B->NS * 8, &d));
        dst = (double *)d;
    }
    HIPCHK(c, launch_unpack(B->g, 24, 1, Fld{(double *)B->Xb.data + (size_t)slot * B->NS, nullptr, P64}, dst,
                            c->stream));
    if (!(flags & SAPDD_DEVICE_PTRS))
        HIPCHK(c, hipMemcpyAsync(x, dst, (size_t)B->NS * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int status = s.status;
    sap_clover_release(B->f, s.kappa, lprec(B->prec));
    s = Slot();  // an elastic slot keeps its memory for the next add (sapdd_batch_trim frees it)
    s.H.assign((size_t)(B->m + 1) * B->m, 0.0);
    s.cs.assign(B->m, 0.0);
    s.sn.assign(B->m, 0.0);
    s.gv.assign(B->m + 1, 0.0);
    if (status == SAPDD_ENAN) return fail(c, SAPDD_ENAN, "non-finite residual in slot %d", slot);
    return SAPDD_OK;
}

// Solve = one batch holding every right-hand side, stepped until all are finished. The
// context keeps the batch between calls with compatible arguments, so repeated solves
// allocate nothing.
int sapdd_solve(sapdd_ctx *c, const sapdd_field *fc, const double *kappa, const sapdd_params *p, int nrhs,
                const double *b, double *x, sapdd_stats *stats) {
    const double t0 = now_s();
    if (!c || !fc || !kappa || !b || !x || !p) return fail(c, SAPDD_EINVAL, "null argument");
    if (nrhs < 1) return fail(c, SAPDD_EINVAL, "nrhs must be >= 1");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_batch *B = c->solve_batch;
    if (batch_reusable(B, fc, p, nrhs)) {
        CHK(batch_release_slots(B));
    } else {
        if (B) batch_free(B);
        c->solve_batch = nullptr;
        sapdd_params q = *p;
        CHK(sapdd_batch_create(c, fc, &q, nrhs, &B));
        c->solve_batch = B;
    }
    return batch_solve_all(B, kappa, p, nrhs, b, x, stats, t0);
}

}  // extern "C"

namespace {

// Add nrhs right-hand sides, step the batch until all finish and take the solutions.
int batch_solve_all(sapdd_batch *B, const double *kappa, const sapdd_params *p, int nrhs, const double *b, double *x,
                    sapdd_stats *stats, double t0) {
    sapdd_ctx *c = B->c;
    B->p.tol = p->tol;
    B->p.max_iter = p->max_iter;
    B->p.gap = p->gap;
    B->t_sap = B->t_d = B->t_gs = B->t_host = 0;
    const size_t NS = (size_t)B->NS;
    std::vector<int> slot(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        CHK(sapdd_batch_add(B, kappa[r], b + r * NS, (p->flags & SAPDD_USE_X0) ? x + r * NS : nullptr,
                            p->flags & SAPDD_DEVICE_PTRS, &slot[r]));
    }
    int running = nrhs;
    while (running > 0) CHK(sapdd_batch_step(B, &running));
    int status = SAPDD_OK;
    const double t1 = now_s();
    for (int r = 0; r < nrhs; ++r) {
        sapdd_stats st;
        const int rc = sapdd_batch_take(B, slot[r], x + r * NS, p->flags & SAPDD_DEVICE_PTRS, &st);
        st.t_total = t1 - t0;
        if (stats) stats[r] = st;
        if (rc != SAPDD_OK) status = rc;
        else if (!st.converged && status == SAPDD_OK) status = SAPDD_ENOCONV;
    }
    if (status == SAPDD_ENOCONV) return fail(c, SAPDD_ENOCONV, "not converged within max_iter = %d", p->max_iter);
    return status;
}

// Colouring for probing D_c: m_mu = the smallest divisor >= 3 of the block-grid extent
// G_mu (G_mu itself if there is none), so two aggregates of one colour are never both
// among an aggregate and its neighbours unless they coincide.
MgColouring mg_colouring(const Geom &g) {
    MgColouring cl{};
    cl.n = 1;
    for (int mu = 0; mu < 4; ++mu) {
        int m = g.G[mu];
        for (int d = 3; d < g.G[mu]; ++d)
            if (g.G[mu] % d == 0) {
                m = d;
                break;
            }
        cl.m[mu] = m;
        cl.n *= m;
    }
    return cl;
}

int mg_alloc(sapdd_mg *mg, size_t bytes, void **out) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        return fail(mg->c, SAPDD_ENOMEM, "hipMalloc of %zu bytes for the multigrid failed", bytes);
    }
    mg->allocs.push_back(q);
    *out = q;
    return SAPDD_OK;
}

void mg_free(sapdd_mg *mg) {
    if (!mg) return;
    if (mg->c) (void)hipStreamSynchronize(mg->c->stream);
    if (mg->batch) batch_free(mg->batch);
    for (void *q : mg->allocs) (void)hipFree(q);
    delete mg;
}

// Copy n doubles from a device buffer to the caller's array (host or device per flags).
int copy_out(sapdd_ctx *c, const void *src, double *dst, size_t n, int flags) {
    HIPCHK(c, hipMemcpyAsync(dst, src, n * 8,
                             (flags & SAPDD_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SAPDD_OK;
}

int mg_setup_body(sapdd_mg *mg, const double *vecs, int flags) {
    sapdd_ctx *c = mg->c;
    sapdd_field *f = mg->f;
    const Geom &g = f->geo;
    const int nvec = mg->nvec, K = mg->K;
    const size_t NS = (size_t)g.V * 24;
    void *q;
    CHK(mg_alloc(mg, (size_t)nvec * NS * sizeof(float), &q));
    mg->P = (float *)q;
    CHK(mg_alloc(mg, (size_t)g.Nd * 9 * K * K * sizeof(float2), &q));
    mg->Dc = (float2 *)q;
    // test vectors into the device layout (FP64)
    const double *src;
    CHK(stage_in(c, "stage_in", vecs, (size_t)nvec * NS, flags, &src));
    CHK(buf(c, "mg_w", (size_t)nvec * NS * 8, &q));
    double *w = (double *)q;
    HIPCHK(c, launch_pack(g, 24, nvec, src, Fld{w, nullptr, P64}, c->stream));
    int *ident;
    CHK(identity_list(c, std::max(nvec, K), &ident));
    if (mg->mp.setup_iters > 0) {  // v <- v - SAP(M v)
        std::vector<double> kap(nvec, mg->kappa);
        SapState s;
        CHK(sap_prepare(c, f, kap.data(), nvec, mg->sp.sap_prec, &s));
        CHK(buf(c, "mg_sm_t", (size_t)nvec * NS * 8, &q));
        double *t = (double *)q;
        CHK(buf(c, "mg_sm_psi", (size_t)nvec * NS * 8, &q));
        double *psi = (double *)q;
        for (int it = 0; it < mg->mp.setup_iters; ++it) {
            DslashIO io{};
            io.in = Fld{w, nullptr, P64};
            io.out = Fld{t, nullptr, P64};
            io.active = ident;
            io.nact = nvec;
            io.in_stride = io.out_stride = io.sub_stride = 1;
            KLAUNCH(c, SAPDD_K_DSLASH, launch_dslash_full(g, links_of(f, P64), tclov_of(f, P64), mg->kappa, io,
                                                          c->stream));
            CHK(sap_run(c, g, s, &mg->sp, t, 1, nullptr, 0, psi, P64, 1, ident, nvec));
            KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_axpy(g, Fld{w, nullptr, P64}, NS, psi, NS, -1.0, nullptr, 0, ident,
                                                       nvec, c->stream));
        }
    }
    KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_orth(g, w, nvec, c->stream));
    HIPCHK(c, launch_convert(g, 24, nvec, w, Fld{mg->P, nullptr, P32}, c->stream));
    // D_c column by column: for every colour and chunk of coarse columns, interpolate the
    // unit vectors, apply the FP64 operator, restrict and scatter into the stencil.
    HIPCHK(c, hipMemsetAsync(mg->Dc, 0, (size_t)g.Nd * 9 * K * K * sizeof(float2), c->stream));
    const int chunk = std::min(K, 16);
    CHK(buf(c, "mg_pr_in", (size_t)chunk * NS * 8, &q));
    double *pin = (double *)q;
    CHK(buf(c, "mg_pr_out", (size_t)chunk * NS * 8, &q));
    double *pout = (double *)q;
    CHK(buf(c, "mg_pr_r", (size_t)chunk * g.Nd * K * sizeof(float2), &q));
    float2 *R = (float2 *)q;
    for (int col = 0; col < mg->cl.n; ++col)
        for (int k0 = 0; k0 < K; k0 += chunk) {
            const int nk = std::min(chunk, K - k0);
            KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_prolong_probe(g, mg->nvec, mg->P, col, mg->cl, k0, nk, pin,
                                                                c->stream));
            DslashIO io{};
            io.in = Fld{pin, nullptr, P64};
            io.out = Fld{pout, nullptr, P64};
            io.active = ident;
            io.nact = nk;
            io.in_stride = io.out_stride = io.sub_stride = 1;
            KLAUNCH(c, SAPDD_K_DSLASH, launch_dslash_full(g, links_of(f, P64), tclov_of(f, P64), mg->kappa, io,
                                                          c->stream));
            KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_restrict(g, mg->nvec, pout, (int64_t)NS, mg->P, R,
                                                           (int64_t)g.Nd * K, nullptr, nk, c->stream));
            KLAUNCH(c, SAPDD_K_MG_FINE, launch_mg_scatter(g, R, nk, k0, K, col, mg->cl, mg->Dc, c->stream));
        }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SAPDD_OK;
}

}  // namespace

extern "C" {

int sapdd_mg_setup(sapdd_ctx *c, sapdd_field *f, double kappa, const sapdd_params *smoother,
                   const sapdd_mg_params *mgp, const double *vecs, int flags, sapdd_mg **out) {
    if (!c || !f || !smoother || !mgp || !vecs || !out) return fail(c, SAPDD_EINVAL, "null argument");
    *out = nullptr;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    CHK(check_params(c, f, smoother));
    if (!(kappa > 0)) return fail(c, SAPDD_EINVAL, "kappa must be > 0");
    if (mgp->nvec < 2 || mgp->nvec > MG_NVEC_MAX || mgp->nvec % 2)
        return fail(c, SAPDD_EINVAL, "nvec must be even and in 2..%d", MG_NVEC_MAX);
    if (mgp->coarse_iters < 1 || mgp->coarse_iters > MG_IMAX)
        return fail(c, SAPDD_EINVAL, "coarse_iters must be in 1..%d", MG_IMAX);
    if (mgp->setup_iters < 0 || mgp->coarse_cycles < 0 || mgp->coarse_cycles > 64)
        return fail(c, SAPDD_EINVAL, "setup_iters must be >= 0 and coarse_cycles in 0..64");
    if (mgp->coarse_form != 0 && mgp->coarse_form != 1) return fail(c, SAPDD_EINVAL, "coarse_form must be 0 or 1");
    const Geom &g = f->geo;
    if (g.Vb > 512) return fail(c, SAPDD_EINVAL, "multigrid aggregates (Schwarz blocks) must have <= 512 sites");
    if ((int64_t)mgp->coarse_iters > g.Nd * 2 * mgp->nvec)
        return fail(c, SAPDD_EINVAL, "coarse_iters exceeds the coarse dimension");
    sapdd_mg *mg = new sapdd_mg;
    mg->c = c;
    mg->f = f;
    mg->kappa = kappa;
    mg->sp = *smoother;
    mg->mp = *mgp;
    mg->nvec = mgp->nvec;
    mg->K = 2 * mgp->nvec;
    mg->cycles = std::max(1, mgp->coarse_cycles);
    mg->cl = mg_colouring(g);
    const int r = mg_setup_body(mg, vecs, flags);
    if (r != SAPDD_OK) {
        mg_free(mg);
        return r;
    }
    *out = mg;
    return SAPDD_OK;
}

int sapdd_mg_destroy(sapdd_mg *mg) {
    mg_free(mg);
    return SAPDD_OK;
}

int sapdd_mg_prolongator(sapdd_mg *mg, double *fields, int flags) {
    if (!mg || !fields) return SAPDD_EINVAL;
    sapdd_ctx *c = mg->c;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    const Geom &g = mg->f->geo;
    const size_t n = (size_t)mg->nvec * g.V * 24;
    void *q;
    CHK(buf(c, "stage_out", n * 8, &q));
    HIPCHK(c, launch_unpack(g, 24, mg->nvec, Fld{mg->P, nullptr, P32}, (double *)q, c->stream));
    return copy_out(c, q, fields, n, flags);
}

int sapdd_mg_coarse_operator(sapdd_mg *mg, double *stencil, int flags) {
    if (!mg || !stencil) return SAPDD_EINVAL;
    sapdd_ctx *c = mg->c;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    const Geom &g = mg->f->geo;
    const int K = mg->K;
    const size_t n = (size_t)g.Nd * 9 * K * K;
    std::vector<float2> h(n);
    HIPCHK(c, hipMemcpyAsync(h.data(), mg->Dc, n * sizeof(float2), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // device: column-major blocks; canonical: row-major blocks, complex128
    std::vector<double> o(2 * n);
    for (size_t blk = 0; blk < (size_t)g.Nd * 9; ++blk)
        for (int row = 0; row < K; ++row)
            for (int col = 0; col < K; ++col) {
                const float2 v = h[(blk * K + col) * K + row];
                o[2 * ((blk * K + row) * K + col)] = v.x;
                o[2 * ((blk * K + row) * K + col) + 1] = v.y;
            }
    if (flags & SAPDD_DEVICE_PTRS) {
        HIPCHK(c, hipMemcpyAsync(stencil, o.data(), 2 * n * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        memcpy(stencil, o.data(), 2 * n * 8);
    }
    return SAPDD_OK;
}

int sapdd_mg_coarse_solve(sapdd_mg *mg, int n, const double *rhs, double *out, int flags) {
    if (!mg || !rhs || !out || n < 1) return SAPDD_EINVAL;
    sapdd_ctx *c = mg->c;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    const Geom &g = mg->f->geo;
    const size_t nc = (size_t)g.Nd * mg->K;
    MgWork w;
    CHK(mg_work_init(mg, n, [&](const char *name, size_t bytes, void **q) { return buf(c, name, bytes, q); }, &w));
    int *ident;
    CHK(identity_list(c, n, &ident));
    const double *src;
    CHK(stage_in(c, "stage_in", rhs, (size_t)n * nc * 2, flags, &src));
    const MgGmres G = mg_gmres(mg, w, ident);
    KLAUNCH(c, SAPDD_K_MG_COARSE, launch_mg_load(G, n, src, (int64_t)nc * 2, c->stream));
    KLAUNCH(c, SAPDD_K_MG_COARSE, launch_mg_coarse_gmres(G, n, mg->mp.coarse_iters, mg->cycles, c->stream));
    void *q;
    CHK(buf(c, "stage_out", (size_t)n * nc * 16, &q));
    KLAUNCH(c, SAPDD_K_MG_COARSE, launch_mg_solution(G, n, (double *)q, (int64_t)nc * 2, c->stream));
    return copy_out(c, q, out, (size_t)n * nc * 2, flags);
}

int sapdd_mg_precond(sapdd_mg *mg, int nrhs, const double *in, double *out, int flags) {
    if (!mg || !in || !out || nrhs < 1) return SAPDD_EINVAL;
    sapdd_ctx *c = mg->c;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_field *f = mg->f;
    const Geom &g = f->geo;
    const size_t NS = (size_t)g.V * 24;
    std::vector<double> kap(nrhs, mg->kappa);
    SapState s;
    CHK(sap_prepare(c, f, kap.data(), nrhs, mg->sp.sap_prec, &s));
    MgWork w;
    CHK(mg_work_init(mg, nrhs, [&](const char *name, size_t bytes, void **q) { return buf(c, name, bytes, q); },
                     &w));
    int *ident;
    CHK(identity_list(c, nrhs, &ident));
    const double *src;
    CHK(stage_in(c, "stage_in", in, (size_t)nrhs * NS, flags, &src));
    void *q;
    CHK(buf(c, "mg_eta", (size_t)nrhs * NS * 8, &q));
    double *eta = (double *)q;
    CHK(buf(c, "mg_psi", (size_t)nrhs * NS * 8, &q));
    double *psi = (double *)q;
    HIPCHK(c, launch_pack(g, 24, nrhs, src, Fld{eta, nullptr, P64}, c->stream));
    CHK(mg_run(c, mg, w, s, &mg->sp, eta, 1, nullptr, 0, psi, P64, 1, ident, nrhs));
    CHK(buf(c, "stage_out", (size_t)nrhs * NS * 8, &q));
    HIPCHK(c, launch_unpack(g, 24, nrhs, Fld{psi, nullptr, P64}, (double *)q, c->stream));
    return copy_out(c, q, out, (size_t)nrhs * NS, flags);
}

int sapdd_batch_set_mg(sapdd_batch *B, sapdd_mg *mg) {
    if (!B || !mg) return SAPDD_EINVAL;
    sapdd_ctx *c = B->c;
    c->err.clear();
    if (mg->f != B->f || mg->c != c) return fail(c, SAPDD_EINVAL, "the multigrid belongs to another field or context");
    if (B->elastic) return fail(c, SAPDD_EINVAL, "an elastic batch cannot precondition with the multigrid");
    for (const auto &s : B->slots)
        if (s.used) return fail(c, SAPDD_EINVAL, "the batch has slots in use");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &kv : B->graphs) (void)hipGraphExecDestroy(kv.second);  // captured for the old preconditioner
    B->graphs.clear();
    CHK(mg_work_init(mg, B->cap, [&](const char *, size_t bytes, void **q) { return balloc(B, bytes, q); }, &B->mw));
    B->mg = mg;
    return SAPDD_OK;
}

int sapdd_mg_solve(sapdd_mg *mg, const sapdd_params *p, int nrhs, const double *b, double *x, sapdd_stats *stats) {
    const double t0 = now_s();
    if (!mg || !p || !b || !x) return SAPDD_EINVAL;
    sapdd_ctx *c = mg->c;
    if (nrhs < 1) return fail(c, SAPDD_EINVAL, "nrhs must be >= 1");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_batch *B = mg->batch;
    if (batch_reusable(B, mg->f, p, nrhs)) {
        CHK(batch_release_slots(B));
    } else {
        if (B) batch_free(B);
        mg->batch = nullptr;
        sapdd_params q = *p;
        CHK(sapdd_batch_create(c, mg->f, &q, nrhs, &B));
        const int r = sapdd_batch_set_mg(B, mg);
        if (r != SAPDD_OK) {
            batch_free(B);
            return r;
        }
        mg->batch = B;
    }
    std::vector<double> kap(nrhs, mg->kappa);
    return batch_solve_all(B, kap.data(), p, nrhs, b, x, stats, t0);
}

}  // extern "C"
