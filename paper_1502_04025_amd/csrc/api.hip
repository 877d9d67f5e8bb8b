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
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/sapdd.h"
#include "kernels.hpp"

using namespace sapdd;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
};

size_t prec_bytes(int prec) { return prec == P64 ? 8 : prec == P32 ? 4 : 2; }

struct XEntry {  // SAP clover X for one (kappa, precision)
    double kappa;
    int prec;
    Fld x;
    unsigned long long last_use;
};

}  // namespace

struct sapdd_field {
    Geom geo;
    double *links64 = nullptr;
    double *tclov64 = nullptr;
    Fld links_lo[3] = {};  // [P32], [P16] lower-precision copies, made on demand
    Fld tclov_lo[3] = {};
    std::vector<XEntry> xcache;
    unsigned long long use_clock = 0;
    double csw = 0.0;
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
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // SAP sweep per (nact, j)
    // kernel profiling: event pairs recorded around launches, drained at sync points
    bool prof = false;
    std::vector<hipEvent_t> pev;
    std::vector<int> pkind;
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
        c->plaunch[c->pkind[i]] += 1;
    }
    c->pn = 0;
    return SAPDD_OK;
}

// Record the start event of a profiled launch of family `kind` (no-op when profiling is off).
int prof_begin(sapdd_ctx *c, int kind) {
    if (!c->prof) return SAPDD_OK;
    if (2 * (c->pn + 1) > c->pev.size()) {
        if (c->pev.size() >= 8192) {  // pool full: wait for the stream and drain it
            HIPCHK(c, hipStreamSynchronize(c->stream));
            int r = prof_drain(c);
            if (r != SAPDD_OK) return r;
        } else {
            const size_t old = c->pev.size();
            c->pev.resize(old ? 2 * old : 256);
            c->pkind.resize(c->pev.size() / 2);
            for (size_t i = old; i < c->pev.size(); ++i) HIPCHK(c, hipEventCreate(&c->pev[i]));
        }
    }
    c->pkind[c->pn] = kind;
    HIPCHK(c, hipEventRecord(c->pev[2 * c->pn], c->stream));
    return SAPDD_OK;
}

int prof_end(sapdd_ctx *c) {
    if (!c->prof) return SAPDD_OK;
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

// SAP clover X for (kappa, prec), cached on the field (a few entries, least recently used out).
int sap_clover(sapdd_ctx *c, sapdd_field *f, double kappa, int prec, Fld *out) {
    for (auto &e : f->xcache)
        if (e.kappa == kappa && e.prec == prec) {
            e.last_use = ++f->use_clock;
            *out = e.x;
            return SAPDD_OK;
        }
    const size_t max_entries = 16;
    if (f->xcache.size() >= max_entries) {
        auto it = std::min_element(f->xcache.begin(), f->xcache.end(),
                                   [](const XEntry &a, const XEntry &b) { return a.last_use < b.last_use; });
        HIPCHK(c, hipStreamSynchronize(c->stream));
        free_fld(it->x);
        f->xcache.erase(it);
    }
    const Geom &g = f->geo;
    XEntry e;
    e.kappa = kappa;
    e.prec = prec;
    e.last_use = ++f->use_clock;
    size_t bytes = (size_t)g.V * 72 * prec_bytes(prec);
    const size_t sc_off = (bytes + 255) / 256 * 256;
    if (prec == P16) bytes = sc_off + (size_t)g.V * sizeof(float);
    void *p = nullptr;
    HIPCHK(c, hipMalloc(&p, bytes));
    e.x = Fld{p, prec == P16 ? (float *)((char *)p + sc_off) : nullptr, prec};
    HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    HIPCHK(c, launch_sap_clover(g, f->tclov64, kappa, e.x, c->d_flag, c->stream));
    int sing = 0;
    HIPCHK(c, hipMemcpyAsync(&sing, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (sing) {
        (void)hipFree(p);
        return fail(c, SAPDD_ESINGULAR, "clover block 1 + kappa T is singular at kappa = %g", kappa);
    }
    f->xcache.push_back(e);
    *out = e.x;
    return SAPDD_OK;
}

int check_params(sapdd_ctx *c, const sapdd_field *f, const sapdd_params *p) {
    if (!p) return fail(c, SAPDD_EINVAL, "params is NULL");
    const bool zero = !p->block[0] && !p->block[1] && !p->block[2] && !p->block[3];
    if (!zero)
        for (int mu = 0; mu < 4; ++mu)
            if (p->block[mu] != f->geo.B[mu])
                return fail(c, SAPDD_EINVAL, "params.block differs from the field's blocking");
    if (p->nmr < 1 || p->ncy < 1) return fail(c, SAPDD_EINVAL, "nmr and ncy must be >= 1");
    if (p->sap_prec < SAPDD_F64 || p->sap_prec > SAPDD_F16) return fail(c, SAPDD_EINVAL, "bad sap_prec");
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

// Upload per-rhs kappa and clover pointers; prepare rres/delta buffers.
int sap_prepare(sapdd_ctx *c, sapdd_field *f, const double *kappa, int nrhs, int prec, SapState *s) {
    const Geom &g = f->geo;
    CHK(lo_copies(c, f, prec));
    s->links = links_of(f, prec);
    std::vector<Fld> xs(nrhs);
    for (int r = 0; r < nrhs; ++r) CHK(sap_clover(c, f, kappa[r], prec, &xs[r]));
    CHK(spinor_buf(c, "sap_rres", g, nrhs, prec, 12, &s->rres));
    CHK(spinor_buf(c, "sap_delta", g, nrhs, prec, 24, &s->delta));
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
    *out = c;
    return SAPDD_OK;
}

void sapdd_destroy(sapdd_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
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
    }
    for (auto &e : f->xcache) free_fld(e.x);
    f->xcache.clear();
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

int sapdd_free_field(sapdd_ctx *c, sapdd_field *f) {
    if (!f) return SAPDD_OK;
    if (c) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
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
    CHK(lo_copies(c, f, prec));
    const double *src;
    CHK(stage_in(c, "stage_in", in, nd, flags, &src));
    Fld fin, fout;
    CHK(spinor_buf(c, "op_in", g, nrhs, prec, 24, &fin));
    CHK(spinor_buf(c, "op_out", g, nrhs, prec, 24, &fout));
    HIPCHK(c, launch_pack(g, 24, nrhs, src, fin, c->stream));
    if (block) {
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

int sapdd_sap(sapdd_ctx *c, const sapdd_field *fc, double kappa, const sapdd_params *p, int nrhs, const double *in,
              double *out) {
    if (!c || !fc || !in || !out) return fail(c, SAPDD_EINVAL, "null argument");
    if (nrhs < 1) return fail(c, SAPDD_EINVAL, "nrhs must be >= 1");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_field *f = const_cast<sapdd_field *>(fc);
    CHK(check_params(c, f, p));
    const Geom &g = f->geo;
    const size_t nd = (size_t)g.V * 24 * nrhs;
    const int prec = p->sap_prec;
    const int psi_prec = prec == P64 ? P64 : P32;
    std::vector<double> kap(nrhs, kappa);
    SapState s;
    CHK(sap_prepare(c, f, kap.data(), nrhs, prec, &s));
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

long long sapdd_solve_footprint(const sapdd_field *f, const sapdd_params *p, int nrhs) {
    if (!f || !p || nrhs < 1) return -1;
    const long long V = f->geo.V;
    const int m = std::max(1, p->restart);
    const int prec = p->sap_prec;
    const long long sb = prec == P64 ? 8 : prec == P32 ? 4 : 2;
    const long long zb = prec == P64 ? 8 : 4;
    long long per_rhs = (m + 1) * V * 24 * 8     // Krylov basis V
                        + (long long)m * V * 24 * zb  // preconditioned vectors Z
                        + 2 * V * 24 * 8              // b and x in the device layout
                        + V * 24 * sb + V * 12 * sb + (prec == P16 ? 2 * V * 4 : 0)  // SAP delta, residual
                        + V * 72 * sb + (prec == P16 ? V * 4 : 0);                     // clover X per kappa
    long long fixed = prec == P64 ? 0 : 2 * V * 72 * sb + (prec == P16 ? 2 * V * 4 : 0);  // low-precision links, T
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

// ====================================================================== FGMRES
namespace {

typedef std::complex<double> cd;

struct RhsState {
    int rhs;
    double bnorm = 0, beta = 0, est = 0, true_relres = 0;
    int iters = 0, restarts = 0, converged = 0, nz = 0;
    bool in_cycle = false;
    bool dirty = false;  // x changed since the last true residual
    std::vector<cd> H;  // (m+1) x m column major: H[i + (m+1) j]
    std::vector<cd> cs, sn, gv;
};

struct Layout {
    int m;
    int CST;  // doubles per rhs in the coefficient block: h[2(m+1)], c[2(m+1)], nrm
    int hoff, coff, noff;
};

// Upload an int list into device segment `seg` of the list pool (pinned staging `host`).
int upload_list(sapdd_ctx *c, int *dpool, int *hpool, int seg, int maxn, const std::vector<int> &v, int **out) {
    for (size_t i = 0; i < v.size(); ++i) hpool[seg * maxn + i] = v[i];
    HIPCHK(c, hipMemcpyAsync(dpool + seg * maxn, hpool + seg * maxn, v.size() * sizeof(int), hipMemcpyHostToDevice,
                             c->stream));
    *out = dpool + seg * maxn;
    return SAPDD_OK;
}

}  // namespace

extern "C" int sapdd_solve(sapdd_ctx *c, const sapdd_field *fc, const double *kappa, const sapdd_params *p, int nrhs,
                           const double *b, double *x, sapdd_stats *stats) {
    const double t0 = now_s();
    if (!c || !fc || !kappa || !b || !x) return fail(c, SAPDD_EINVAL, "null argument");
    if (nrhs < 1) return fail(c, SAPDD_EINVAL, "nrhs must be >= 1");
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    sapdd_field *f = const_cast<sapdd_field *>(fc);
    CHK(check_params(c, f, p));
    // the fused correct-and-dot Gram-Schmidt pass holds all basis vectors of a step at once
    if (p->restart < 1 || p->restart > 16) return fail(c, SAPDD_EINVAL, "restart must be in 1..16");
    if (!(p->tol > 0) || p->max_iter < 1) return fail(c, SAPDD_EINVAL, "tol must be > 0 and max_iter >= 1");
    for (int r = 0; r < nrhs; ++r)
        if (!(kappa[r] > 0)) return fail(c, SAPDD_EINVAL, "kappa must be > 0");
    const Geom &g = f->geo;
    const int m = p->restart;
    const int prec = p->sap_prec;
    const int zprec = prec == P64 ? P64 : P32;
    const int64_t NS = g.V * 24;  // doubles per spinor field
    const int64_t ncx = g.V * 12; // complex entries per field
    const int flags = p->flags;
    const size_t nd = (size_t)NS * nrhs;

    // ---- buffers
    Fld Vb, Zb, Bb, Xb;
    CHK(spinor_buf(c, "kry_V", g, nrhs * (m + 1), P64, 24, &Vb));
    CHK(spinor_buf(c, "kry_Z", g, nrhs * m, zprec, 24, &Zb));
    CHK(spinor_buf(c, "kry_b", g, nrhs, P64, 24, &Bb));
    CHK(spinor_buf(c, "kry_x", g, nrhs, P64, 24, &Xb));
    double *Vd = (double *)Vb.data, *Bd = (double *)Bb.data, *Xd = (double *)Xb.data;
    SapState ss;
    CHK(sap_prepare(c, f, kappa, nrhs, prec, &ss));
    Layout L;
    L.m = m;
    L.hoff = 0;
    L.coff = 2 * (m + 1);
    L.noff = 4 * (m + 1);
    L.CST = 4 * (m + 1) + 2;
    const int nwg_d = dslash_full_partials(g);
    const int nwg_b = std::max(blas_partials(ncx, nrhs), blas_partials(ncx, 1));
    const int maxval = 32;
    double *coef, *vscale, *part, *ydev;
    {
        void *q;
        CHK(buf(c, "kry_coef", (size_t)nrhs * L.CST * 8, &q));
        coef = (double *)q;
        CHK(buf(c, "kry_vscale", (size_t)nrhs * (m + 1) * 8, &q));
        vscale = (double *)q;
        CHK(buf(c, "kry_part", (size_t)nrhs * std::max(nwg_d, nwg_b * maxval) * 8, &q));
        part = (double *)q;
        CHK(buf(c, "kry_y", (size_t)nrhs * 2 * m * 8, &q));
        ydev = (double *)q;
    }
    const int nseg = 8;
    int *dlists;
    {
        void *q;
        CHK(buf(c, "kry_lists", (size_t)nseg * nrhs * sizeof(int), &q));
        dlists = (int *)q;
    }
    const size_t pin_bytes = (size_t)nseg * nrhs * sizeof(int) + (size_t)nrhs * L.CST * 8 + (size_t)nrhs * 2 * m * 8;
    void *pin;
    CHK(pinned(c, pin_bytes, &pin));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int *hlists = (int *)pin;
    double *hcoef = (double *)((char *)pin + (size_t)nseg * nrhs * sizeof(int));
    double *hy = hcoef + (size_t)nrhs * L.CST;
    double *dkappa = ss.kappa;

    // ---- inputs into the device layout
    const double *bsrc;
    CHK(stage_in(c, "stage_in", b, nd, flags, &bsrc));
    HIPCHK(c, launch_pack(g, 24, nrhs, bsrc, Bb, c->stream));
    if (flags & SAPDD_USE_X0) {
        const double *xsrc;
        CHK(stage_in(c, "stage_in2", x, nd, flags, &xsrc));
        HIPCHK(c, launch_pack(g, 24, nrhs, xsrc, Xb, c->stream));
    } else {
        HIPCHK(c, hipMemsetAsync(Xd, 0, nd * 8, c->stream));
    }

    std::vector<RhsState> st(nrhs);
    std::vector<int> all(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        all[r] = r;
        st[r].rhs = r;
        st[r].H.assign((size_t)(m + 1) * m, 0.0);
        st[r].cs.assign(m, 0.0);
        st[r].sn.assign(m, 0.0);
        st[r].gv.assign(m + 1, 0.0);
    }
    int *d_all;
    CHK(upload_list(c, dlists, hlists, 0, nrhs, all, &d_all));
    // |b| per rhs
    {
        CgsArgs a{};
        a.w = Bd;
        a.wstride = NS;
        a.part = part;
        a.active = d_all;
        a.nact = nrhs;
        a.nv = 0;
        a.n = ncx;
        KLAUNCH(c, SAPDD_K_GS, launch_cgs(2, a, c->stream));
        KLAUNCH(c, SAPDD_K_GS, launch_reduce(part, blas_partials(ncx, nrhs), 1, d_all, nrhs, coef + L.noff, L.CST, nullptr, 0, 0,
                                nullptr, 0, c->stream));
        HIPCHK(c, hipMemcpyAsync(hcoef, coef, (size_t)nrhs * L.CST * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int r = 0; r < nrhs; ++r) st[r].bnorm = std::sqrt(hcoef[(size_t)r * L.CST + L.noff]);
    }

    double t_sap = 0, t_d = 0, t_gs = 0, t_host = 0;
    int status = SAPDD_OK;
    std::vector<int> active;  // rhs still unconverged
    for (int r = 0; r < nrhs; ++r) {
        if (st[r].bnorm == 0.0) {
            st[r].converged = 1;  // x = 0 solves b = 0
        } else {
            active.push_back(r);
        }
    }

    while (!active.empty()) {
        int *d_act;
        CHK(upload_list(c, dlists, hlists, 1, nrhs, active, &d_act));
        const int nact = (int)active.size();
        // ---- true residual r = b - M x into basis slot 0, |r|^2, vscale[0] = 1/|r|
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        DslashIO io{};
        io.in = Xb;
        io.out = Fld{Vd, nullptr, P64};
        io.sub = Bd;
        io.part = part;
        io.active = d_act;
        io.nact = nact;
        io.in_stride = 1;
        io.out_stride = m + 1;
        io.sub_stride = 1;
        io.kappa = dkappa;
        KLAUNCH(c, SAPDD_K_DSLASH, launch_dslash_full(g, links_of(f, P64), tclov_of(f, P64), 0.0, io, c->stream));
        KLAUNCH(c, SAPDD_K_GS, launch_reduce(part, nwg_d, 1, d_act, nact, coef + L.noff, L.CST, nullptr, 0, 0, vscale, m + 1,
                                c->stream));
        HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
        HIPCHK(c, hipMemcpyAsync(hcoef, coef, (size_t)nrhs * L.CST * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->prof) CHK(prof_drain(c));
        {
            float ms;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
            t_d += ms * 1e-3;
        }
        std::vector<int> cycle;
        for (int r : active) {
            RhsState &s = st[r];
            s.dirty = false;
            s.beta = std::sqrt(hcoef[(size_t)r * L.CST + L.noff]);
            s.true_relres = s.beta / s.bnorm;
            if (!std::isfinite(s.beta)) {
                status = fail(c, SAPDD_ENAN, "non-finite residual for rhs %d", r);
                continue;
            }
            if (s.true_relres <= p->tol) {
                s.converged = 1;
                continue;
            }
            if (s.iters >= p->max_iter) continue;
            cycle.push_back(r);
        }
        if (status != SAPDD_OK) break;
        // unconverged rhs out of iterations leave the active set
        std::vector<int> next_active;
        for (int r : active)
            if (!st[r].converged && st[r].iters < p->max_iter) next_active.push_back(r);
        active = next_active;
        if (cycle.empty()) break;
        for (int r : cycle) {
            RhsState &s = st[r];
            std::fill(s.H.begin(), s.H.end(), 0.0);
            std::fill(s.gv.begin(), s.gv.end(), 0.0);
            s.gv[0] = s.beta;
            s.in_cycle = true;
            s.nz = 0;
        }
        int *d_cyc;
        CHK(upload_list(c, dlists, hlists, 2, nrhs, cycle, &d_cyc));
        int ncyc = (int)cycle.size();
        for (int j = 0; j < m && ncyc > 0; ++j) {
            // ---- z_j = SAP(v_j)
            HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
            CHK(sap_run(c, g, ss, p, Vd + (size_t)j * NS, m + 1, vscale + j, m + 1,
                        (char *)Zb.data + (size_t)j * NS * prec_bytes(zprec), zprec, m, d_cyc, ncyc));
            HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
            // ---- w = M z_j into basis slot j + 1
            DslashIO w{};
            w.in = Fld{(char *)Zb.data + (size_t)j * NS * prec_bytes(zprec), nullptr, zprec};
            w.out = Fld{Vd + (size_t)(j + 1) * NS, nullptr, P64};
            w.active = d_cyc;
            w.nact = ncyc;
            w.in_stride = m;
            w.out_stride = m + 1;
            w.kappa = dkappa;
            KLAUNCH(c, SAPDD_K_DSLASH, launch_dslash_full(g, links_of(f, P64), tclov_of(f, P64), 0.0, w, c->stream));
            HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
            // ---- CGS2 against v_0 .. v_j
            CgsArgs a{};
            a.vbase = Vd;
            a.vstride = NS;
            a.rstride = (int64_t)(m + 1) * NS;
            a.vscale = vscale;
            a.vsstride = m + 1;
            a.w = Vd + (size_t)(j + 1) * NS;
            a.wstride = (int64_t)(m + 1) * NS;
            a.cstride = L.CST;
            a.part = part;
            a.active = d_cyc;
            a.nact = ncyc;
            a.n = ncx;
                const int nwg = blas_partials(ncx, ncyc);
            for (int pass = 0; pass < 2; ++pass) {
                // pass 0: h = V^H w (then w -= V h in the next launch); pass 1: c = V^H w'
                const int outoff = pass == 0 ? L.hoff : L.coff;
                for (int v0 = 0; v0 <= j; v0 += 16) {
                    a.v0 = v0;
                    a.nv = std::min(16, j + 1 - v0);
                    if (pass == 0) {
                        KLAUNCH(c, SAPDD_K_GS, launch_cgs(0, a, c->stream));
                    } else {
                        a.coef = coef + L.hoff;
                        KLAUNCH(c, SAPDD_K_GS, launch_cgs(1, a, c->stream));
                    }
                    KLAUNCH(c, SAPDD_K_GS, launch_reduce(part, nwg, 2 * a.nv, d_cyc, ncyc, coef + outoff + 2 * v0, L.CST, vscale,
                                            m + 1, v0, nullptr, 0, c->stream));
                }
            }
            // w'' = w' - V c, |w''|^2, vscale[j+1] = 1/|w''|
            a.coef = coef + L.coff;
            a.v0 = 0;
            a.nv = j + 1;
            KLAUNCH(c, SAPDD_K_GS, launch_cgs(2, a, c->stream));
            KLAUNCH(c, SAPDD_K_GS, launch_reduce(part, nwg, 1, d_cyc, ncyc, coef + L.noff, L.CST, nullptr, 0, 0, vscale + j + 1,
                                    m + 1, c->stream));
            HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
            HIPCHK(c, hipMemcpyAsync(hcoef, coef, (size_t)nrhs * L.CST * 8, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (c->prof) CHK(prof_drain(c));
            const double th = now_s();
            {
                float ms;
                HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
                t_sap += ms * 1e-3;
                HIPCHK(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
                t_d += ms * 1e-3;
                HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
                t_gs += ms * 1e-3;
            }
            // ---- host: Hessenberg column, Givens rotation, residual estimate
            std::vector<int> still;
            for (int r : cycle) {
                RhsState &s = st[r];
                if (!s.in_cycle) continue;
                const double *hc = hcoef + (size_t)r * L.CST;
                cd *col = &s.H[(size_t)(m + 1) * j];
                for (int i = 0; i <= j; ++i)
                    col[i] = cd(hc[L.hoff + 2 * i] + hc[L.coff + 2 * i], hc[L.hoff + 2 * i + 1] + hc[L.coff + 2 * i + 1]);
                const double hn = std::sqrt(std::max(0.0, hc[L.noff]));
                col[j + 1] = hn;
                for (int i = 0; i < j; ++i) {  // previous rotations
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
                if (!std::isfinite(s.est)) {
                    status = fail(c, SAPDD_ENAN, "non-finite Arnoldi coefficients for rhs %d", r);
                    s.in_cycle = false;
                    continue;
                }
                if (s.est <= p->tol || hn == 0.0 || den == 0.0 || s.iters >= p->max_iter) {
                    s.in_cycle = false;
                    continue;
                }
                still.push_back(r);
            }
            t_host += now_s() - th;
            if (status != SAPDD_OK) break;
            if (still.size() != (size_t)ncyc) {
                cycle = still;
                ncyc = (int)cycle.size();
                if (ncyc) CHK(upload_list(c, dlists, hlists, 2 + ((j + 1) % 2), nrhs, cycle, &d_cyc));
            }
        }
        if (status != SAPDD_OK) break;
        // ---- x += Z y for every rhs that took part in this cycle, grouped by basis size
        std::map<int, std::vector<int>> groups;
        for (int r : all)
            if (st[r].nz > 0) groups[st[r].nz].push_back(r);
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int seg = 4;
        for (auto &kv : groups) {
            const int nz = kv.first;
            for (int r : kv.second) {
                RhsState &s = st[r];
                // back substitution R y = g
                std::vector<cd> y(nz);
                for (int i = nz - 1; i >= 0; --i) {
                    cd t = s.gv[i];
                    for (int k = i + 1; k < nz; ++k) t -= s.H[(size_t)(m + 1) * k + i] * y[k];
                    const cd d = s.H[(size_t)(m + 1) * i + i];
                    y[i] = d != 0.0 ? t / d : 0.0;
                }
                for (int i = 0; i < nz; ++i) {
                    hy[(size_t)r * 2 * m + 2 * i] = y[i].real();
                    hy[(size_t)r * 2 * m + 2 * i + 1] = y[i].imag();
                }
                s.restarts += 1;
                s.nz = 0;
                s.dirty = true;
            }
        }
        HIPCHK(c, hipMemcpyAsync(ydev, hy, (size_t)nrhs * 2 * m * 8, hipMemcpyHostToDevice, c->stream));
        for (auto &kv : groups) {
            int *d_grp;
            CHK(upload_list(c, dlists, hlists, seg, nrhs, kv.second, &d_grp));
            seg = seg + 1 < nseg ? seg + 1 : 4;
            KLAUNCH(c, SAPDD_K_UPDATE, launch_zupdate(Xd, NS, Zb.data, zprec, NS, (int64_t)m * NS, ydev, 2 * m, kv.first, d_grp,
                                     (int)kv.second.size(), ncx, g.Vbh, c->stream));
            if (seg == 4) HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }

    // ---- final true residuals for the record (rhs that stopped without a final check)
    {
        std::vector<int> chk;
        for (int r = 0; r < nrhs; ++r)
            if (st[r].bnorm > 0 && st[r].dirty) chk.push_back(r);
        if (!chk.empty()) {
            int *d_chk;
            CHK(upload_list(c, dlists, hlists, 1, nrhs, chk, &d_chk));
            DslashIO io{};
            io.in = Xb;
            io.out = Fld{Vd, nullptr, P64};
            io.sub = Bd;
            io.part = part;
            io.active = d_chk;
            io.nact = (int)chk.size();
            io.in_stride = 1;
            io.out_stride = m + 1;
            io.sub_stride = 1;
            io.kappa = dkappa;
            KLAUNCH(c, SAPDD_K_DSLASH, launch_dslash_full(g, links_of(f, P64), tclov_of(f, P64), 0.0, io, c->stream));
            KLAUNCH(c, SAPDD_K_GS, launch_reduce(part, nwg_d, 1, d_chk, io.nact, coef + L.noff, L.CST, nullptr, 0, 0, nullptr, 0,
                                    c->stream));
            HIPCHK(c, hipMemcpyAsync(hcoef, coef, (size_t)nrhs * L.CST * 8, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            for (int r : chk) {
                st[r].true_relres = std::sqrt(hcoef[(size_t)r * L.CST + L.noff]) / st[r].bnorm;
                st[r].converged = st[r].true_relres <= p->tol;
                st[r].dirty = false;
            }
        }
    }
    // ---- x back to the canonical layout
    double *dst = x;
    if (!(flags & SAPDD_DEVICE_PTRS)) {
        void *d;
        CHK(buf(c, "stage_out", nd * 8, &d));
        dst = (double *)d;
    }
    HIPCHK(c, launch_unpack(g, 24, nrhs, Xb, dst, c->stream));
    if (!(flags & SAPDD_DEVICE_PTRS)) HIPCHK(c, hipMemcpyAsync(x, dst, nd * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double t1 = now_s();
    bool all_conv = true;
    for (int r = 0; r < nrhs; ++r) {
        all_conv = all_conv && st[r].converged;
        if (stats) {
            sapdd_stats &o = stats[r];
            o.iters = st[r].iters;
            o.restarts = st[r].restarts;
            o.converged = st[r].converged;
            o.true_relres = st[r].true_relres;
            o.implicit_relres = st[r].est;
            o.t_total = t1 - t0;
            o.t_sap = t_sap;
            o.t_dslash = t_d;
            o.t_gs = t_gs;
            o.t_host = t_host;
        }
    }
    if (status != SAPDD_OK) return status;
    if (!all_conv) return fail(c, SAPDD_ENOCONV, "not converged within max_iter = %d", p->max_iter);
    return SAPDD_OK;
}
