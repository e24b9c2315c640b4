// C ABI of the GRPIC hot path (declared in include/grpic.h): handle state,
// allocation, the per-step driver and the host<->device copies, for the FP64
// form and the FP32-mixed form.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/grpic.h"
#include "grpic_dev.h"
#include "grpic_impl.h"

using namespace grpic;

// Staging area of grpic_load_particles_noalloc: the host arrays of one call
// (positions and covariant velocities, 6 doubles per particle) are copied
// here before the load kernel reads them.  Each device the library runs on
// holds its own copy of the array, at its own address, until the process
// ends.  Host code never uses the array's name as an address: the device
// address comes from hipGetSymbolAddress, once per device (noalloc_staging).
constexpr int64_t kNoAllocLoadMax = (int64_t)1 << 20;  // particles per call (48 MiB)
static __device__ __align__(256) double scratch[6 * kNoAllocLoadMax];

struct grpic_s {
    grpic_config cfg;
    bool mixed;  // FP32-mixed form
    hipStream_t stream;
    int device;               // device current at creation
    double *noalloc_staging;  // that device's address of `scratch` (NULL: not resolved)
    Grid G;
    Hole h;
    Species S;
    Mixed M;
    FieldPtrsT<double> F64;
    FieldPtrsT<float> F32;
    // FP64 particles
    double *px[2][3];
    double *pu[2][4];
    // FP32-mixed particles
    int32_t *pcell[2];
    float *poff[2][3];
    float *pu32[2][4];
    uint8_t *psp[2];
    int xc, uc;
    int64_t n_slots, cap;
    unsigned long long *counters;
    double jscale, rscale;
    uint32_t *keys, *keys_alt, *idx, *idx_alt;
    void *sort_temp;
    int key_bits;
    unsigned long long *rho_scratch;
    double *red;
    int64_t red_cap;
    std::vector<void *> allocs;
    int64_t step_count;
    int sticky;
    // C_FLAGS as last copied to the host (pinned; written by an asynchronous
    // copy at the end of every grpic_step call)
    volatile unsigned long long *flags_host;
    // the kernels of one cycle captured as a graph per buffer parity
    // (xc, uc), each for the slot count it was captured with
    int use_graphs;
    hipGraphExec_t cycle_exec[2][2];
    int64_t cycle_slots[2][2];
    // the run created its stream itself (the caller passed the null stream)
    bool own_stream;
    // event timing
    int timing;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[GRPIC_NTIMERS];
};

namespace {

int check_at(hipError_t e, const char *what, int line) {
    if (e == hipSuccess) return GRPIC_OK;
    fprintf(stderr, "grpic: %s failed at api.hip:%d: HIP error %d (%s)\n", what, line, (int)e, hipGetErrorString(e));
    return GRPIC_EDEVICE;
}
#define check(e) check_at((e), #e, __LINE__)
#define FAILS(e) (check_at((e), #e, __LINE__) != GRPIC_OK)

// Errors left by earlier HIP calls of the host program (not this library)
// must not be reported as ours: clear them on entry.
void clear_foreign_error() { (void)hipGetLastError(); }

// Device address of `scratch` on device dev, resolved once per device with
// that device current (the caller's current device when a run is created).
constexpr int kMaxDevices = 64;
std::mutex g_staging_mu;
double *g_staging[kMaxDevices] = {};

double *noalloc_staging(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_staging_mu);
    if (!g_staging[dev]) {
        void *p = nullptr;
        if (FAILS(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))) return nullptr;
        g_staging[dev] = (double *)p;
    }
    return g_staging[dev];
}

void *raw_alloc(grpic_t *h, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (h->cfg.alloc) {
        p = h->cfg.alloc(bytes, h->cfg.alloc_ctx);
    } else if (FAILS(hipMalloc(&p, bytes))) {
        p = nullptr;
    }
    if (!p) fprintf(stderr, "grpic: device allocation of %zu bytes failed\n", bytes);
    return p;
}

void raw_free(grpic_t *h, void *p) {
    if (!p) return;
    if (h->cfg.alloc) {
        if (h->cfg.free) h->cfg.free(p, h->cfg.alloc_ctx);
    } else {
        (void)hipFree(p);
    }
}

void *dev_alloc(grpic_t *h, size_t bytes) {
    void *p = raw_alloc(h, bytes);
    if (p) h->allocs.push_back(p);
    return p;
}

// Scratch device buffer for one call (freed after the stream drained).
struct Temp {
    grpic_t *h;
    void *p;
    Temp(grpic_t *hh, size_t bytes) : h(hh), p(raw_alloc(hh, bytes)) {}
    ~Temp() {
        if (p) {
            (void)hipStreamSynchronize(h->stream);
            raw_free(h, p);
        }
    }
};

hipEvent_t take_event(grpic_t *h) {
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (FAILS(hipEventCreate(&e))) return nullptr;
    return e;
}

// Bracket a kernel group with events when timing is on.
struct TimedGroup {
    grpic_t *h;
    int t;
    hipEvent_t a, b;
    TimedGroup(grpic_t *hh, int tt) : h(hh), t(tt), a(nullptr), b(nullptr) {
        if (!h->timing) return;
        a = take_event(h);
        b = take_event(h);
        if (a) (void)hipEventRecord(a, h->stream);
    }
    ~TimedGroup() {
        if (!h->timing || !a || !b) return;
        (void)hipEventRecord(b, h->stream);
        h->ev_used[t].push_back({a, b});
    }
};

ParticlePtrs pp(grpic_t *h, int xb, int ub) {
    ParticlePtrs P;
    for (int q = 0; q < 3; q++) P.x[q] = h->px[xb][q];
    for (int q = 0; q < 4; q++) P.u[q] = h->pu[ub][q];
    P.sp = h->psp[ub];
    return P;
}

ParticlePtrs32 pp32(grpic_t *h, int xb, int ub) {
    ParticlePtrs32 P;
    P.cell = h->pcell[xb];
    for (int q = 0; q < 3; q++) P.off[q] = h->poff[xb][q];
    for (int q = 0; q < 4; q++) P.u[q] = h->pu32[ub][q];
    P.sp = h->psp[ub];
    return P;
}

template <typename T> FieldPtrsT<T> &fields(grpic_t *h);
template <> FieldPtrsT<double> &fields<double>(grpic_t *h) { return h->F64; }
template <> FieldPtrsT<float> &fields<float>(grpic_t *h) { return h->F32; }

int validate(const grpic_config *c) {
    if (!c) return GRPIC_EINVAL;
    if (c->nx < 4 || c->ny < 4 || c->nz < 4) return GRPIC_EINVAL;
    if (c->nx > 1020 || c->ny > 1020 || c->nz > 1020) return GRPIC_EINVAL;  // packed cells hold 10 bits
    if ((int64_t)c->nx * c->ny * c->nz > (int64_t)1 << 30) return GRPIC_EINVAL;
    if (c->precision != GRPIC_FP64 && c->precision != GRPIC_FP32_MIXED) return GRPIC_EINVAL;
    if (c->gamma_mode != GRPIC_GAMMA_PAPER && c->gamma_mode != GRPIC_GAMMA_U4) return GRPIC_EINVAL;
    if (c->deposit_mode != GRPIC_DEPOSIT_CURVED && c->deposit_mode != GRPIC_DEPOSIT_FLAT) return GRPIC_EINVAL;
    if (c->rk_mode != GRPIC_RK_CLASSIC && c->rk_mode != GRPIC_RK_PRINTED) return GRPIC_EINVAL;
    if (c->gather_mode != GRPIC_GATHER_STAGE && c->gather_mode != GRPIC_GATHER_STEP) return GRPIC_EINVAL;
    if (c->gather_weights != GRPIC_WEIGHTS_TRILINEAR && c->gather_weights != GRPIC_WEIGHTS_SPATIAL)
        return GRPIC_EINVAL;
    // the push ablations exist in the FP64 pusher only
    if (c->precision != GRPIC_FP64 && (c->rk_mode != GRPIC_RK_CLASSIC || c->gather_mode != GRPIC_GATHER_STAGE ||
                                       c->gather_weights != GRPIC_WEIGHTS_TRILINEAR))
        return GRPIC_EINVAL;
    if (c->field_iters < 1 || c->field_iters > 16) return GRPIC_EINVAL;
    if (c->sort_every < 0 || c->tile < 1 || c->tile > 64) return GRPIC_EINVAL;
    if (c->fp_bits < 16 || c->fp_bits > 50) return GRPIC_EINVAL;
    if (c->nspecies < 1 || c->nspecies > GRPIC_MAX_SPECIES) return GRPIC_EINVAL;
    if (!(c->c > 0.0) || !(c->dt > 0.0) || !isfinite(c->c) || !isfinite(c->dt)) return GRPIC_EINVAL;
    // Courant condition of the 3D Yee scheme with unit cells
    if (!(c->c * c->dt < 1.0 / sqrt(3.0))) return GRPIC_EINVAL;
    if (!(c->m >= 0.0) || !(fabs(c->a) <= c->m) || !isfinite(c->m)) return GRPIC_EINVAL;
    if (c->m > 0.0 && !(c->r_exc >= 0.0 && c->r_exc < c->r_rm)) return GRPIC_EINVAL;
    if (c->damp_max < 0.0 || c->damp_max > 1.0) return GRPIC_EINVAL;
    if (!(c->outer_layer >= 0.0) || !isfinite(c->outer_layer) || !(c->outer_damp >= 0.0) || c->outer_damp > 1.0)
        return GRPIC_EINVAL;
    for (int s = 0; s < c->nspecies; s++) {
        if (!(c->mass[s] > 0.0) || !isfinite(c->mass[s]) || !isfinite(c->charge[s])) return GRPIC_EINVAL;
        // plasma-frequency criterion (Sec. 5.1): omega_p dt < 2 with
        // omega_p^2 = 4 pi n q^2 / m at the species' nominal density n
        // (macro-particles per unit cell volume; 0: not checked).  Its
        // general-relativistic form gamma^(-1/2) omega_p dt < 2 follows for
        // every gamma >= 1.
        const double n = c->density[s];
        if (!(n >= 0.0) || !isfinite(n)) return GRPIC_EINVAL;
        if (n > 0.0 && !(sqrt(4.0 * M_PI * n * c->charge[s] * c->charge[s] / c->mass[s]) * c->dt < 2.0))
            return GRPIC_EINVAL;
    }
    if (c->capacity < 0 || c->capacity > ((int64_t)1 << 31) - 1) return GRPIC_EINVAL;
    return GRPIC_OK;
}

template <typename T>
bool alloc_fields(grpic_t *h, FieldPtrsT<T> &F) {
    int64_t gs = h->G.gsize(), nn = h->G.nnodes();
    bool ok = true;
    auto A = [&](size_t bytes) -> void * {
        void *p = dev_alloc(h, bytes);
        if (!p) ok = false;
        return p;
    };
    for (int c = 0; c < 3; c++) {
        F.D[c] = (T *)A(gs * sizeof(T));
        F.B[c] = (T *)A(gs * sizeof(T));
        F.E[c] = (T *)A(gs * sizeof(T));
        F.H[c] = (T *)A(gs * sizeof(T));
        F.D0[c] = (T *)A(gs * sizeof(T));
        F.B0[c] = (T *)A(gs * sizeof(T));
        F.E0[c] = (T *)A(gs * sizeof(T));
        F.H0[c] = (T *)A(gs * sizeof(T));
        F.Dsave[c] = (T *)A(gs * sizeof(T));
        F.Bsave[c] = (T *)A(gs * sizeof(T));
        F.Jint[c] = (unsigned long long *)A(gs * 8);
    }
    F.rho_abs = (unsigned long long *)A(gs * 8);
    F.mask = (uint8_t *)A(gs);
    F.w = (T *)A(6 * nn * sizeof(T));
    F.node = (T *)A(16 * nn * sizeof(T));
    return ok;
}

template <typename T>
int init_fields(grpic_t *h, FieldPtrsT<T> &F) {
    hipStream_t s = h->stream;
    int64_t gs = h->G.gsize();
    int rc = GRPIC_OK;
    for (int c = 0; c < 3 && !rc; c++) {
        if (FAILS(hipMemsetAsync(F.E[c], 0, gs * sizeof(T), s))) rc = GRPIC_EDEVICE;
        if (FAILS(hipMemsetAsync(F.H[c], 0, gs * sizeof(T), s))) rc = GRPIC_EDEVICE;
        if (FAILS(hipMemsetAsync(F.Jint[c], 0, gs * 8, s))) rc = GRPIC_EDEVICE;
    }
    if (!rc && FAILS(hipMemsetAsync(F.rho_abs, 0, gs * 8, s))) rc = GRPIC_EDEVICE;
    if (rc) return rc;
    launch_bake<T>(h->G, h->h, F, s);
    launch_init_fields<T>(h->G, h->h, F, h->cfg.B0, h->cfg.init_covariant, s);
    // reference state: evolved values and their derived fields at t = 0
    for (int c = 0; c < 3; c++) {
        if (FAILS(hipMemcpyAsync(F.D0[c], F.D[c], gs * sizeof(T), hipMemcpyDeviceToDevice, s))) return GRPIC_EDEVICE;
        if (FAILS(hipMemcpyAsync(F.B0[c], F.B[c], gs * sizeof(T), hipMemcpyDeviceToDevice, s))) return GRPIC_EDEVICE;
    }
    launch_derived<T>(h->G, h->h, F, false, true, true, s);
    for (int c = 0; c < 3; c++) {
        if (FAILS(hipMemcpyAsync(F.E0[c], F.E[c], gs * sizeof(T), hipMemcpyDeviceToDevice, s))) return GRPIC_EDEVICE;
        if (FAILS(hipMemcpyAsync(F.H0[c], F.H[c], gs * sizeof(T), hipMemcpyDeviceToDevice, s))) return GRPIC_EDEVICE;
    }
    return GRPIC_OK;
}

// Magnetic half-step to time n with E_cov^n made consistent with B^n, then
// the node tensor from (D^n, B^n).
template <typename T>
int fields_to_n(grpic_t *h) {
    FieldPtrsT<T> &F = fields<T>(h);
    const grpic_config &c = h->cfg;
    hipStream_t s = h->stream;
    TimedGroup tg(h, GRPIC_TIMER_FIELDS);
    launch_save<T>(h->G, F, 0, s);
    const T *Bsave[3] = {F.Bsave[0], F.Bsave[1], F.Bsave[2]};
    for (int it = 0; it < c.field_iters; it++) {
        launch_derived<T>(h->G, h->h, F, true, true, false, s);
        launch_bhalf<T>(h->G, F, Bsave, 0.5 * c.c * c.dt, s);
    }
    launch_node_tensor<T>(h->G, h->h, F, s);
    return GRPIC_OK;
}

// Second magnetic half-step (same E_cov^n) and clearing of the current.
template <typename T>
void fields_mid(grpic_t *h) {
    FieldPtrsT<T> &F = fields<T>(h);
    TimedGroup tg(h, GRPIC_TIMER_FIELDS);
    const T *Bcur[3] = {F.B[0], F.B[1], F.B[2]};
    launch_bhalf<T>(h->G, F, Bcur, 0.5 * h->cfg.c * h->cfg.dt, h->stream);
    launch_zero3_u64(F.Jint, h->G.gsize(), h->stream);
}

// Electric step around D^{n+1/2}, then the relaxation layer.
template <typename T>
int fields_d(grpic_t *h) {
    FieldPtrsT<T> &F = fields<T>(h);
    const grpic_config &c = h->cfg;
    hipStream_t s = h->stream;
    TimedGroup tg(h, GRPIC_TIMER_FIELDS);
    launch_save<T>(h->G, F, 1, s);
    const T *Dsave[3] = {F.Dsave[0], F.Dsave[1], F.Dsave[2]};
    double inv_js = 1.0 / h->jscale;
    double fpc = 4.0 * M_PI / c.c;
    for (int it = 0; it < c.field_iters; it++) {
        launch_derived<T>(h->G, h->h, F, true, false, true, s);
        double dtp = (it < c.field_iters - 1) ? 0.5 * c.dt : c.dt;
        launch_dstep<T>(h->G, F, Dsave, c.c * dtp, fpc, inv_js, s);
    }
    launch_relax<T>(h->G, h->h, F, c.r_damp, c.damp_max, s);
    launch_relax_outer<T>(h->G, F, c.outer_layer, c.outer_damp, s);
    return GRPIC_OK;
}

PushParams push_params(grpic_t *h) {
    PushParams P;
    P.G = h->G;
    P.h = h->h;
    P.c = h->cfg.c;
    P.dt = h->cfg.dt;
    P.inv_c = 1.0 / h->cfg.c;
    P.dt_2c = h->cfg.dt / (2.0 * h->cfg.c);
    P.dt_6 = h->cfg.dt / 6.0;
    P.gamma_mode = h->cfg.gamma_mode;
    P.rk_mode = h->cfg.rk_mode;
    P.gather_mode = h->cfg.gather_mode;
    P.gather_weights = h->cfg.gather_weights;
    P.n = h->n_slots;
    return P;
}

void push_particles(grpic_t *h) {
    TimedGroup tg(h, GRPIC_TIMER_PUSH);
    PushParams P = push_params(h);
    if (h->mixed)
        launch_push32(P, h->M, h->S, h->F32.node, pp32(h, h->xc, h->uc), pp32(h, 1 - h->xc, h->uc), h->counters,
                      h->stream);
    else
        launch_push(P, h->S, h->F64.node, pp(h, h->xc, h->uc), pp(h, 1 - h->xc, h->uc), h->counters, h->stream);
}

void deposit_particles(grpic_t *h) {
    TimedGroup tg(h, GRPIC_TIMER_DEPOSIT);
    const grpic_config &c = h->cfg;
    if (h->mixed)
        launch_deposit32(h->G, h->h, h->M, c.dt, c.deposit_mode, c.r_rm, h->jscale, h->rscale, h->S,
                         pp32(h, h->xc, h->uc), pp32(h, 1 - h->xc, h->uc), h->n_slots, h->F32, h->counters,
                         h->stream);
    else
        launch_deposit(h->G, h->h, c.dt, c.deposit_mode, c.r_rm, h->jscale, h->rscale, h->S, pp(h, h->xc, h->uc),
                       pp(h, 1 - h->xc, h->uc), h->n_slots, h->F64, h->counters, h->stream);
}

// keep: leave the sorted keys and the permutation for grpic_sort.
int do_sort(grpic_t *h, bool keep = false, uint32_t **final_keys = nullptr, uint32_t **final_idx = nullptr) {
    TimedGroup tg(h, GRPIC_TIMER_SORT);
    if (h->mixed)
        launch_sort32(h->G, h->cfg.tile, h->n_slots, pp32(h, h->xc, h->uc), pp32(h, 1 - h->xc, 1 - h->uc), h->keys,
                      h->keys_alt, h->idx, h->idx_alt, h->sort_temp, h->key_bits, keep, final_keys, final_idx,
                      h->counters, h->stream);
    else
        launch_sort(h->G, h->cfg.tile, h->n_slots, pp(h, h->xc, h->uc), pp(h, 1 - h->xc, 1 - h->uc), h->keys,
                    h->keys_alt, h->idx, h->idx_alt, h->sort_temp, h->key_bits, keep, final_keys, final_idx,
                    h->counters, h->stream);
    h->xc = 1 - h->xc;
    h->uc = 1 - h->uc;
    return check(hipGetLastError());
}

// The kernels of one cycle (everything but the cell sort), enqueued on the
// run's stream.
template <typename T>
int cycle_kernels(grpic_t *h) {
    int rc = fields_to_n<T>(h);
    if (rc) return rc;
    push_particles(h);
    fields_mid<T>(h);
    deposit_particles(h);
    return fields_d<T>(h);
}

int cycle_kernels(grpic_t *h) { return h->mixed ? cycle_kernels<float>(h) : cycle_kernels<double>(h); }

void drop_cycle_graphs(grpic_t *h) {
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            if (h->cycle_exec[a][b]) (void)hipGraphExecDestroy(h->cycle_exec[a][b]);
            h->cycle_exec[a][b] = nullptr;
        }
}

// The captured cycle of the current buffer parity and slot count, captured
// now if there is none (the launches' pointers and grid sizes depend only on
// them; the configuration and the buffers are fixed for the run).
int cycle_graph(grpic_t *h, hipGraphExec_t *out) {
    hipGraphExec_t &ex = h->cycle_exec[h->xc][h->uc];
    if (ex && h->cycle_slots[h->xc][h->uc] == h->n_slots) {
        *out = ex;
        return GRPIC_OK;
    }
    if (ex) (void)hipGraphExecDestroy(ex);
    ex = nullptr;
    int rc = check(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    if (rc) return rc;
    int krc = cycle_kernels(h);
    hipGraph_t g = nullptr;
    rc = check(hipStreamEndCapture(h->stream, &g));
    if (!rc) rc = krc;
    if (!rc) rc = check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    if (g) (void)hipGraphDestroy(g);
    if (rc) {
        ex = nullptr;
        return rc;
    }
    h->cycle_slots[h->xc][h->uc] = h->n_slots;
    *out = ex;
    return GRPIC_OK;
}

// One cycle: the captured graph of its kernels when graphs are on and no
// kernel is being timed (the timing brackets each kernel group with events
// recorded per launch), else the kernels launched one by one; then the cell
// sort when it is due.
int one_step(grpic_t *h, bool allow_sort = true) {
    int rc;
    if (h->use_graphs && !h->timing && h->stream) {
        hipGraphExec_t ex = nullptr;
        rc = cycle_graph(h, &ex);
        if (!rc) rc = check(hipGraphLaunch(ex, h->stream));
    } else {
        rc = cycle_kernels(h);
    }
    if (rc) return rc;
    h->xc = 1 - h->xc;
    h->step_count++;
    if (allow_sort && h->cfg.sort_every > 0 && h->step_count % h->cfg.sort_every == 0) return do_sort(h);
    return check(hipGetLastError());
}

// The cell sort of grpic_step falls due at the end of the next cycle.
bool sort_due_after_cycle(const grpic_t *h) {
    return h->cfg.sort_every > 0 && (h->step_count + 1) % h->cfg.sort_every == 0;
}

// FP64 view of the particle state (the FP32-mixed form is widened into
// tmp, which must hold 7 n doubles).
ParticlePtrs f64_view(grpic_t *h, double *tmp) {
    if (!h->mixed) return pp(h, h->xc, h->uc);
    int64_t n = h->n_slots;
    launch_to_f64(pp32(h, h->xc, h->uc), tmp, tmp + 3 * n, n, h->stream);
    ParticlePtrs P;
    for (int q = 0; q < 3; q++) P.x[q] = tmp + q * n;
    for (int q = 0; q < 4; q++) P.u[q] = tmp + (3 + q) * n;
    P.sp = h->psp[h->uc];
    return P;
}

template <typename T>
int copy_field_out(grpic_t *h, const T *src, double *out, int64_t count) {
    if (sizeof(T) == sizeof(double)) {
        int rc = check(hipMemcpyAsync(out, src, count * 8, hipMemcpyDeviceToHost, h->stream));
        return rc ? rc : check(hipStreamSynchronize(h->stream));
    }
    std::vector<T> tmp(count);
    int rc = check(hipMemcpyAsync(tmp.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, h->stream));
    if (!rc) rc = check(hipStreamSynchronize(h->stream));
    for (int64_t i = 0; i < count && !rc; i++) out[i] = (double)tmp[i];
    return rc;
}

template <typename T>
int copy_field_in(grpic_t *h, T *dst, const double *in, int64_t count) {
    if (sizeof(T) == sizeof(double)) {
        int rc = check(hipMemcpyAsync(dst, in, count * 8, hipMemcpyHostToDevice, h->stream));
        return rc ? rc : check(hipStreamSynchronize(h->stream));
    }
    std::vector<T> tmp(count);
    for (int64_t i = 0; i < count; i++) tmp[i] = (T)in[i];
    int rc = check(hipMemcpyAsync(dst, tmp.data(), count * sizeof(T), hipMemcpyHostToDevice, h->stream));
    if (!rc) rc = check(hipStreamSynchronize(h->stream));
    return rc;
}

template <typename T>
int dump_fields_t(grpic_t *h, int which, double *out) {
    FieldPtrsT<T> &F = fields<T>(h);
    int64_t gs = h->G.gsize();
    int rc = GRPIC_OK;
    if (which == 4) {
        std::vector<long long> tmp(gs);
        for (int q = 0; q < 3 && !rc; q++) {
            rc = check(hipMemcpyAsync(tmp.data(), F.Jint[q], gs * 8, hipMemcpyDeviceToHost, h->stream));
            if (!rc) rc = check(hipStreamSynchronize(h->stream));
            for (int64_t i = 0; i < gs && !rc; i++) out[q * gs + i] = (double)tmp[i] / h->jscale;
        }
        return rc;
    }
    for (int q = 0; q < 3 && !rc; q++) {
        T *src = which == 0 ? F.D[q] : which == 1 ? F.B[q] : which == 2 ? F.E[q] : F.H[q];
        rc = copy_field_out<T>(h, src, out + q * gs, gs);
    }
    return rc;
}

template <typename T>
int restore_fields_t(grpic_t *h, const double *D, const double *B) {
    FieldPtrsT<T> &F = fields<T>(h);
    int64_t gs = h->G.gsize();
    int rc = GRPIC_OK;
    for (int q = 0; q < 3 && !rc; q++) {
        rc = copy_field_in<T>(h, F.D[q], D + q * gs, gs);
        if (!rc) rc = copy_field_in<T>(h, F.B[q], B + q * gs, gs);
    }
    return rc;
}

// Device bytes of a run, mirroring the allocations of grpic_create plus the
// load staging (admission estimate of the batch).
int64_t run_bytes(const grpic_config *c) {
    auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    int64_t gs = (int64_t)(c->nx + 3) * (c->ny + 3) * (c->nz + 3);
    int64_t nn = (int64_t)(c->nx + 1) * (c->ny + 1) * (c->nz + 1);
    int64_t T = c->precision == GRPIC_FP32_MIXED ? 4 : 8;
    int64_t cap = c->capacity > 0 ? c->capacity : 1;
    int64_t b = 0;
    b += 30 * up(gs * T) + 3 * up(gs * 8) + up(gs * 8) + up(gs);
    b += up(6 * nn * T) + up(16 * nn * T);
    if (c->precision == GRPIC_FP32_MIXED)
        b += 2 * (up(cap * 4) + 3 * up(cap * 4) + 4 * up(cap * 4) + up(cap));
    else
        b += 2 * (3 * up(cap * 8) + 4 * up(cap * 8) + up(cap));
    b += up(kCounterWords * 8) + 4 * up(cap * 4) + up((int64_t)sort_temp_bytes(cap)) + up(gs * 8);
    b += up((((cap + 255) / 256) * 12 + ((nn + 255) / 256) * 3 + 64) * 8);
    b += up(7 * cap * 8);  // staging of a particle load or restore
    return b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Serving batch (FP32-mixed runs).  Every iteration rewrites the run table in
// device memory (one host-to-device copy from a pinned double buffer) and
// replays one captured graph of persistent batched launches that advance
// every active run by one cycle; cell sorts that fall due run per run after
// the replay, and finished runs are reduced and freed.
struct BatchRun {
    int64_t id;
    grpic_t *h;                // NULL while preempted or finished
    grpic_config cfg;          // as submitted, to re-create the run on resume
    int32_t nsteps, done, state;
    int64_t bytes;
    grpic_diag diag;
    bool keep;
    int64_t n_slots;
    int64_t particle_steps;
    std::vector<double> x, u;
    std::vector<uint8_t> sp;
};

struct grpic_batch_s {
    int64_t budget, used;
    int32_t max_slots;
    int64_t next_id;
    hipStream_t stream;
    BatchTable *d_table;       // device
    BatchTable *h_table[2];    // pinned host staging, used in turn
    hipEvent_t copied[2];      // the copy out of h_table[k] has completed
    bool copy_pending[2];
    int ring;
    // captured iterations, per (fixed-point passes, radix passes of the
    // sorts that fall due; 0: none)
    std::map<std::pair<int, int>, hipGraphExec_t> execs;
    std::vector<BatchRun *> active;
    std::map<int64_t, BatchRun *> runs;
};

namespace {

// Persistent grids: blocks per CU that the kernels' registers and LDS allow,
// times the 256 compute units.
constexpr int kBatchGridField = 256 * 8;
constexpr int kBatchGridPush = 256 * 4;
constexpr int kBatchGridDep = 256 * 3;

void fill_table_entry(grpic_t *h, BatchRun32 &R) {
    const grpic_config &c = h->cfg;
    R.G = h->G;
    R.h = h->h;
    R.F = h->F32;
    R.hstep = (float)(0.5 * c.c * c.dt);
    R.c = c.c;
    R.dt = c.dt;
    R.fpc = (float)(4.0 * M_PI / c.c);
    R.inv_jscale = 1.0 / h->jscale;
    R.field_iters = c.field_iters;
    relax_box_of(h->G, h->h, c.r_damp, c.damp_max, R.relax_box);
    R.r_damp = c.r_damp;
    R.damp_max = c.damp_max;
    R.P = push_params(h);
    R.M = h->M;
    R.S = h->S;
    R.cur = pp32(h, h->xc, h->uc);
    R.nxt = pp32(h, 1 - h->xc, h->uc);
    R.counters = h->counters;
    R.D = make_dep32(h->G, h->h, h->M, c.dt, c.deposit_mode, h->jscale);
    R.r_rm = c.r_rm;
    R.rscale = h->rscale;
}

// Enqueue one batched iteration (captured into a graph by the caller): the
// cycle of every active run, then the sorts of the runs whose sort falls due
// at the end of this cycle (up to sort_passes radix passes).
void enqueue_iteration(grpic_batch_t *b, int iters, int sort_passes) {
    const BatchTable *T = b->d_table;
    hipStream_t s = b->stream;
    launch_batch_field(BF_SAVE_B, T, 0, kBatchGridField, s);
    for (int it = 0; it < iters; it++) {
        launch_batch_field(BF_NODE_W, T, it, kBatchGridField, s);
        launch_batch_field(BF_ECOV, T, it, kBatchGridField, s);
        launch_batch_field(BF_BHALF_SAVED, T, it, kBatchGridField, s);
    }
    launch_batch_field(BF_NODE_TENSOR, T, 0, kBatchGridField, s);
    launch_batch_push32(T, kBatchGridPush, s);
    launch_batch_field(BF_BHALF_CUR, T, 0, kBatchGridField, s);
    launch_batch_field(BF_ZERO_J, T, 0, kBatchGridField, s);
    launch_batch_deposit32(T, kBatchGridDep, s);
    launch_batch_field(BF_SAVE_D, T, 0, kBatchGridField, s);
    for (int it = 0; it < iters; it++) {
        launch_batch_field(BF_NODE_W, T, it, kBatchGridField, s);
        launch_batch_field(BF_HFIELD, T, it, kBatchGridField, s);
        launch_batch_field(BF_DSTEP, T, it, kBatchGridField, s);
    }
    launch_batch_field(BF_RELAX, T, 0, kBatchGridField, s);
    launch_batch_sort(T, sort_passes, s);
}

// The captured iteration for (iters, sort_passes), captured now if new.
int iteration_graph(grpic_batch_t *b, int iters, int sort_passes, hipGraphExec_t *out) {
    const auto key = std::make_pair(iters, sort_passes);
    auto it = b->execs.find(key);
    if (it != b->execs.end()) {
        *out = it->second;
        return GRPIC_OK;
    }
    int rc = check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    if (rc) return rc;
    enqueue_iteration(b, iters, sort_passes);
    hipGraph_t g = nullptr;
    rc = check(hipStreamEndCapture(b->stream, &g));
    hipGraphExec_t ex = nullptr;
    if (!rc) rc = check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    if (g) (void)hipGraphDestroy(g);
    if (rc) return rc;
    b->execs[key] = ex;
    *out = ex;
    return GRPIC_OK;
}

int finish_run(grpic_batch_t *b, BatchRun *r) {
    grpic_t *h = r->h;
    int rc = grpic_diagnostics(h, &r->diag);
    // a fixed-point overflow is reported in the run's diagnostics (flags bit 1)
    if (rc == GRPIC_EOVERFLOW) rc = GRPIC_OK;
    if (!rc) rc = grpic_particle_steps(h, &r->particle_steps);
    if (!rc && r->keep) {
        r->n_slots = h->n_slots;
        r->x.resize(3 * r->n_slots);
        r->u.resize(4 * r->n_slots);
        r->sp.resize(r->n_slots);
        rc = grpic_dump_particles(h, r->x.data(), r->u.data(), r->sp.data());
    }
    grpic_destroy(h);
    r->h = nullptr;
    b->used -= r->bytes;
    r->state = GRPIC_RUN_DONE;
    return rc;
}

}  // namespace

extern "C" {

int64_t grpic_run_bytes(const grpic_config *cfg) { return cfg ? run_bytes(cfg) : 0; }

int grpic_batch_create(int64_t budget_bytes, int32_t max_slots, grpic_batch_t **out) {
    clear_foreign_error();
    if (!out || budget_bytes <= 0 || max_slots < 1 || max_slots > kMaxBatchRuns) return GRPIC_EINVAL;
    grpic_batch_t *b = new (std::nothrow) grpic_batch_s();
    if (!b) return GRPIC_ENOMEM;
    b->budget = budget_bytes;
    b->max_slots = max_slots;
    b->next_id = 1;
    int rc = GRPIC_OK;
    if (FAILS(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking))) rc = GRPIC_EDEVICE;
    if (!rc && FAILS(hipMalloc((void **)&b->d_table, sizeof(BatchTable)))) rc = GRPIC_ENOMEM;
    for (int k = 0; k < 2 && !rc; k++) {
        if (FAILS(hipHostMalloc((void **)&b->h_table[k], sizeof(BatchTable), hipHostMallocDefault))) rc = GRPIC_ENOMEM;
        if (!rc && FAILS(hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming))) rc = GRPIC_EDEVICE;
    }
    if (rc) {
        grpic_batch_destroy(b);
        return rc;
    }
    *out = b;
    return GRPIC_OK;
}

int grpic_batch_submit(grpic_batch_t *b, const grpic_config *cfg, int32_t nsteps, int32_t keep_state,
                       const int64_t *n, const double *const *x, const double *const *ucov, int64_t *run_id) {
    clear_foreign_error();
    if (!b || !cfg || nsteps < 1 || !n || !x || !ucov || !run_id) return GRPIC_EINVAL;
    if (cfg->alloc || cfg->precision != GRPIC_FP32_MIXED) return GRPIC_EINVAL;
    // the batched stage launches carry no outer absorbing layer
    if (cfg->outer_layer > 0.0 && cfg->outer_damp > 0.0) return GRPIC_EINVAL;
    int rc = validate(cfg);
    if (rc) return rc;
    int64_t bytes = run_bytes(cfg);
    if ((int32_t)b->active.size() >= b->max_slots || b->used + bytes > b->budget) return GRPIC_EAGAIN;
    BatchRun *r = new (std::nothrow) BatchRun();
    if (!r) return GRPIC_ENOMEM;
    rc = grpic_create(cfg, b->stream, &r->h);
    for (int s = 0; s < cfg->nspecies && !rc; s++) rc = grpic_load_particles(r->h, s, n[s], x[s], ucov[s], nullptr);
    if (rc) {
        if (r->h) grpic_destroy(r->h);
        delete r;
        return rc;
    }
    r->id = b->next_id++;
    r->cfg = *cfg;
    r->nsteps = nsteps;
    r->done = 0;
    r->state = GRPIC_RUN_ACTIVE;
    r->bytes = bytes;
    r->keep = keep_state != 0;
    r->n_slots = 0;
    b->used += bytes;
    b->active.push_back(r);
    b->runs[r->id] = r;
    *run_id = r->id;
    return GRPIC_OK;
}

int grpic_batch_step(grpic_batch_t *b, int32_t *finished) {
    clear_foreign_error();
    if (!b) return GRPIC_EINVAL;
    if (finished) *finished = 0;
    if (b->active.empty()) return GRPIC_OK;
    // run table of this iteration, staged in the host buffer whose previous
    // copy has completed
    const int k = b->ring;
    if (b->copy_pending[k] && FAILS(hipEventSynchronize(b->copied[k]))) return GRPIC_EDEVICE;
    BatchTable *T = b->h_table[k];
    const int nr = (int)b->active.size();
    T->nruns = nr;
    int64_t off[BK_NKINDS] = {};
    int iters = 1, sort_passes = 0;
    for (int i = 0; i < nr; i++) {
        grpic_t *h = b->active[i]->h;
        BatchRun32 &R = T->run[i];
        fill_table_entry(h, R);
        // the sort that falls due at the end of this cycle (as in
        // grpic_step): it reads the cycle's output buffers and writes the
        // other pair
        if (sort_due_after_cycle(h)) {
            batch_sort_job(h->G, h->cfg.tile, h->n_slots, pp32(h, 1 - h->xc, h->uc), pp32(h, h->xc, 1 - h->uc),
                           h->keys, h->keys_alt, h->idx, h->idx_alt, h->sort_temp, h->key_bits, R.sort);
            sort_passes = R.sort.passes > sort_passes ? R.sort.passes : sort_passes;
        } else {
            R.sort = BatchSort{};
        }
        for (int kd = 0; kd < BK_NKINDS; kd++) {
            R.off[kd] = off[kd];
            off[kd] += kd >= BK_SORT_SLOT ? batch_sort_blocks(kd, R.sort) : batch_blocks(kd, h->G, R.relax_box, h->n_slots);
        }
        iters = h->cfg.field_iters > iters ? h->cfg.field_iters : iters;
    }
    for (int kd = 0; kd < BK_NKINDS; kd++) T->total[kd] = off[kd];
    const size_t bytes = offsetof(BatchTable, run) + (size_t)nr * sizeof(BatchRun32);
    int rc = check(hipMemcpyAsync(b->d_table, T, bytes, hipMemcpyHostToDevice, b->stream));
    if (!rc) rc = check(hipEventRecord(b->copied[k], b->stream));
    if (rc) return rc;
    b->copy_pending[k] = true;
    b->ring = 1 - k;
    hipGraphExec_t ex = nullptr;
    rc = iteration_graph(b, iters, sort_passes, &ex);
    if (rc) return rc;
    rc = check(hipGraphLaunch(ex, b->stream));
    if (rc) return rc;
    for (BatchRun *r : b->active) {
        grpic_t *h = r->h;
        const bool sorted = sort_due_after_cycle(h);
        h->xc = 1 - h->xc;
        h->step_count++;
        if (sorted) {
            h->xc = 1 - h->xc;
            h->uc = 1 - h->uc;
        }
        r->done++;
    }
    std::vector<BatchRun *> still;
    for (BatchRun *r : b->active) {
        if (r->done >= r->nsteps) {
            int frc = finish_run(b, r);
            if (frc && !rc) rc = frc;
            if (finished) (*finished)++;
        } else {
            still.push_back(r);
        }
    }
    b->active.swap(still);
    return rc;
}

int grpic_batch_poll(grpic_batch_t *b, int64_t run_id, int32_t *state, int32_t *steps_done, grpic_diag *diag,
                     int64_t *n_slots, int64_t *particle_steps) {
    if (!b) return GRPIC_EINVAL;
    auto it = b->runs.find(run_id);
    if (it == b->runs.end()) {
        if (state) *state = GRPIC_RUN_UNKNOWN;
        return GRPIC_OK;
    }
    BatchRun *r = it->second;
    if (state) *state = r->state;
    if (steps_done) *steps_done = r->done;
    if (diag && r->state == GRPIC_RUN_DONE) *diag = r->diag;
    if (n_slots) *n_slots = r->state == GRPIC_RUN_DONE ? r->n_slots : 0;
    if (particle_steps) *particle_steps = r->state == GRPIC_RUN_DONE ? r->particle_steps : 0;
    return GRPIC_OK;
}

int grpic_batch_dump(grpic_batch_t *b, int64_t run_id, double *x, double *u, uint8_t *sp) {
    if (!b) return GRPIC_EINVAL;
    auto it = b->runs.find(run_id);
    if (it == b->runs.end() || it->second->state != GRPIC_RUN_DONE || !it->second->keep) return GRPIC_ESTATE;
    BatchRun *r = it->second;
    if (x) memcpy(x, r->x.data(), r->x.size() * sizeof(double));
    if (u) memcpy(u, r->u.data(), r->u.size() * sizeof(double));
    if (sp) memcpy(sp, r->sp.data(), r->sp.size());
    return GRPIC_OK;
}

int grpic_batch_release(grpic_batch_t *b, int64_t run_id) {
    if (!b) return GRPIC_EINVAL;
    auto it = b->runs.find(run_id);
    if (it == b->runs.end()) return GRPIC_EINVAL;
    if (it->second->state != GRPIC_RUN_DONE && it->second->state != GRPIC_RUN_PREEMPTED) return GRPIC_ESTATE;
    delete it->second;
    b->runs.erase(it);
    return GRPIC_OK;
}

int64_t grpic_batch_state_bytes(grpic_batch_t *b, int64_t run_id) {
    if (!b) return GRPIC_EINVAL;
    auto it = b->runs.find(run_id);
    if (it == b->runs.end()) return GRPIC_EINVAL;
    if (it->second->state != GRPIC_RUN_ACTIVE) return GRPIC_ESTATE;
    return grpic_state_bytes(it->second->h);
}

int grpic_batch_preempt(grpic_batch_t *b, int64_t run_id, void *buf, int64_t bytes) {
    clear_foreign_error();
    if (!b) return GRPIC_EINVAL;
    auto it = b->runs.find(run_id);
    if (it == b->runs.end()) return GRPIC_EINVAL;
    BatchRun *r = it->second;
    if (r->state != GRPIC_RUN_ACTIVE) return GRPIC_ESTATE;
    // the save waits for the batch's stream, so no queued launch still
    // reads the run's memory when it is freed below
    int rc = grpic_save_state(r->h, buf, bytes);
    if (rc) return rc;
    grpic_destroy(r->h);
    r->h = nullptr;
    b->used -= r->bytes;
    r->state = GRPIC_RUN_PREEMPTED;
    b->active.erase(std::find(b->active.begin(), b->active.end(), r));
    return GRPIC_OK;
}

int grpic_batch_resume(grpic_batch_t *b, int64_t run_id, const void *buf, int64_t bytes) {
    clear_foreign_error();
    if (!b) return GRPIC_EINVAL;
    auto it = b->runs.find(run_id);
    if (it == b->runs.end()) return GRPIC_EINVAL;
    BatchRun *r = it->second;
    if (r->state != GRPIC_RUN_PREEMPTED) return GRPIC_ESTATE;
    if ((int32_t)b->active.size() >= b->max_slots || b->used + r->bytes > b->budget) return GRPIC_EAGAIN;
    grpic_t *h = nullptr;
    int rc = grpic_create(&r->cfg, b->stream, &h);
    if (!rc) rc = grpic_load_state(h, buf, bytes);
    // the state must be one of this configuration, taken after the cycles the
    // run has done
    if (!rc && h->step_count != r->done) rc = GRPIC_EINVAL;
    if (rc) {
        if (h) grpic_destroy(h);
        return rc;
    }
    r->h = h;
    r->state = GRPIC_RUN_ACTIVE;
    b->used += r->bytes;
    b->active.push_back(r);
    return GRPIC_OK;
}

int grpic_batch_stats(grpic_batch_t *b, int32_t *active, int64_t *bytes_in_use) {
    if (!b) return GRPIC_EINVAL;
    if (active) *active = (int32_t)b->active.size();
    if (bytes_in_use) *bytes_in_use = b->used;
    return GRPIC_OK;
}

void grpic_batch_destroy(grpic_batch_t *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (BatchRun *r : b->active)
        if (r->h) grpic_destroy(r->h);
    for (auto &kv : b->execs) (void)hipGraphExecDestroy(kv.second);
    for (int k = 0; k < 2; k++) {
        if (b->h_table[k]) (void)hipHostFree(b->h_table[k]);
        if (b->copied[k]) (void)hipEventDestroy(b->copied[k]);
    }
    if (b->d_table) (void)hipFree(b->d_table);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    for (auto &kv : b->runs) delete kv.second;
    delete b;
}

void grpic_config_default(grpic_config *cfg, int32_t nx, int32_t ny, int32_t nz) {
    memset(cfg, 0, sizeof(*cfg));
    cfg->nx = nx;
    cfg->ny = ny;
    cfg->nz = nz;
    cfg->precision = GRPIC_FP64;
    cfg->gamma_mode = GRPIC_GAMMA_PAPER;
    cfg->deposit_mode = GRPIC_DEPOSIT_CURVED;
    cfg->field_iters = 3;
    cfg->sort_every = 10;
    cfg->tile = 4;
    cfg->fp_bits = 44;
    cfg->nspecies = 1;
    cfg->c = 1.0;
    cfg->dt = 0.5;
    cfg->center[0] = nx / 2.0;
    cfg->center[1] = ny / 2.0;
    cfg->center[2] = nz / 2.0;
    cfg->r_rm = 0.0;
    cfg->r_exc = 0.0;
    cfg->r_damp = 0.0;
    cfg->damp_max = 0.1;
    cfg->charge[0] = -1.0;
    cfg->mass[0] = 1.0;
}

size_t grpic_config_size(void) { return sizeof(grpic_config); }

int grpic_config_check(const grpic_config *cfg) { return validate(cfg); }

const char *grpic_strerror(int code) {
    switch (code) {
    case GRPIC_OK: return "ok";
    case GRPIC_EINVAL: return "invalid argument";
    case GRPIC_ENOMEM: return "out of memory or capacity";
    case GRPIC_EDEVICE: return "HIP error";
    case GRPIC_EOVERFLOW: return "fixed-point overflow";
    case GRPIC_ESTATE: return "invalid state";
    case GRPIC_EAGAIN: return "no free slot or memory";
    default: return "unknown error";
    }
}

void grpic_destroy(grpic_t *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    drop_cycle_graphs(h);
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    for (int t = 0; t < GRPIC_NTIMERS; t++)
        for (auto &pr : h->ev_used[t]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (void *p : h->allocs) raw_free(h, p);
    if (h->flags_host) (void)hipHostFree((void *)h->flags_host);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int grpic_create(const grpic_config *cfg, void *stream, grpic_t **out) {
    clear_foreign_error();
    if (!out) return GRPIC_EINVAL;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    grpic_t *h = new (std::nothrow) grpic_s();
    if (!h) return GRPIC_ENOMEM;
    h->cfg = *cfg;
    h->mixed = cfg->precision == GRPIC_FP32_MIXED;
    h->stream = (hipStream_t)stream;
    if (FAILS(hipGetDevice(&h->device))) {
        delete h;
        return GRPIC_EDEVICE;
    }
    if (!h->stream) {
        // a stream of the run's own, blocking (ordered with the null stream
        // both ways) and at the default priority, so the cycle can be
        // captured as a graph while the caller keeps the null stream's order
        if (FAILS(hipStreamCreate(&h->stream))) {
            delete h;
            return GRPIC_EDEVICE;
        }
        h->own_stream = true;
    }
    h->noalloc_staging = noalloc_staging(h->device);
    h->G.nx = cfg->nx;
    h->G.ny = cfg->ny;
    h->G.nz = cfg->nz;
    h->G.sx = cfg->nx + 3;
    h->G.sy = (int64_t)(cfg->ny + 3) * (cfg->nx + 3);
    h->h.m = cfg->m;
    h->h.a = cfg->a;
    h->h.cx = cfg->center[0];
    h->h.cy = cfg->center[1];
    h->h.cz = cfg->center[2];
    h->h.r_exc = cfg->r_exc;
    // FP64 metric and Christoffel symbols within 4 m of the horizon
    // at least 1.25 r_exc, so every excision decision of the FP32-mixed
    // deposit is taken on the FP64 radius
    h->M.r_fp64 = fmax(cfg->m + sqrt(fmax(cfg->m * cfg->m - cfg->a * cfg->a, 0.0)) + 4.0 * cfg->m, 1.25 * cfg->r_exc);
    double qmax = 0.0;
    for (int s = 0; s < kMaxSpecies; s++) {
        bool on = s < cfg->nspecies;
        h->S.charge[s] = on ? cfg->charge[s] : 0.0;
        h->S.mass[s] = on ? cfg->mass[s] : 1.0;
        h->S.qm[s] = on ? cfg->charge[s] / cfg->mass[s] : 0.0;
        if (on && fabs(cfg->charge[s]) > qmax) qmax = fabs(cfg->charge[s]);
    }
    if (qmax == 0.0) qmax = 1.0;
    h->rscale = ldexp(1.0, cfg->fp_bits) / qmax;
    h->jscale = ldexp(1.0, cfg->fp_bits) * cfg->dt / qmax;
    h->cap = cfg->capacity;
    h->use_graphs = 1;

    const Grid &G = h->G;
    int64_t gs = G.gsize(), nn = G.nnodes();
    bool ok = h->mixed ? alloc_fields<float>(h, h->F32) : alloc_fields<double>(h, h->F64);
    auto A = [&](size_t bytes) -> void * {
        void *p = dev_alloc(h, bytes);
        if (!p) ok = false;
        return p;
    };
    int64_t cap = h->cap > 0 ? h->cap : 1;
    for (int b = 0; b < 2; b++) {
        if (h->mixed) {
            h->pcell[b] = (int32_t *)A(cap * 4);
            for (int q = 0; q < 3; q++) h->poff[b][q] = (float *)A(cap * 4);
            for (int q = 0; q < 4; q++) h->pu32[b][q] = (float *)A(cap * 4);
        } else {
            for (int q = 0; q < 3; q++) h->px[b][q] = (double *)A(cap * 8);
            for (int q = 0; q < 4; q++) h->pu[b][q] = (double *)A(cap * 8);
        }
        h->psp[b] = (uint8_t *)A(cap);
    }
    h->counters = (unsigned long long *)A(kCounterWords * 8);
    h->keys = (uint32_t *)A(cap * 4);
    h->keys_alt = (uint32_t *)A(cap * 4);
    h->idx = (uint32_t *)A(cap * 4);
    h->idx_alt = (uint32_t *)A(cap * 4);
    h->sort_temp = A(sort_temp_bytes(cap));
    h->rho_scratch = (unsigned long long *)A(gs * 8);
    h->red_cap = ((cap + 255) / 256) * 12 + ((nn + 255) / 256) * 3 + 64;
    h->red = (double *)A(h->red_cap * 8);
    void *fh = nullptr;
    if (FAILS(hipHostMalloc(&fh, 8, hipHostMallocDefault)))
        ok = false;
    else
        *(unsigned long long *)fh = 0ull;
    h->flags_host = (volatile unsigned long long *)fh;
    if (!ok) {
        grpic_destroy(h);
        return GRPIC_ENOMEM;
    }
    int nTx = (cfg->nx + cfg->tile - 1) / cfg->tile, nTy = (cfg->ny + cfg->tile - 1) / cfg->tile,
        nTz = (cfg->nz + cfg->tile - 1) / cfg->tile;
    uint64_t maxkey = (uint64_t)nTx * nTy * nTz * cfg->tile * cfg->tile * cfg->tile;  // sentinel must exceed it
    int kb = 1;
    while (kb < 32 && (((uint64_t)1 << kb) - 1) <= maxkey) kb++;
    h->key_bits = kb;

    hipStream_t s = h->stream;
    rc = GRPIC_OK;
    if (FAILS(hipMemsetAsync(h->counters, 0, kCounterWords * 8, s))) rc = GRPIC_EDEVICE;
    for (int b = 0; b < 2 && !rc; b++)
        if (FAILS(hipMemsetAsync(h->psp[b], GRPIC_DEAD, cap, s))) rc = GRPIC_EDEVICE;
    if (!rc) rc = h->mixed ? init_fields<float>(h, h->F32) : init_fields<double>(h, h->F64);
    if (!rc) rc = check(hipGetLastError());
    if (!rc) rc = check(hipStreamSynchronize(s));
    if (rc) {
        grpic_destroy(h);
        return rc;
    }
    *out = h;
    return GRPIC_OK;
}

namespace {
// Load through the device staging buffer st (6 n doubles): copy the host
// arrays in, run the load kernel, count the kept particles.  Synchronous.
int load_staged(grpic_t *h, int32_t species, int64_t n, const double *x, const double *ucov, int64_t *kept,
                double *st) {
    hipStream_t s = h->stream;
    int rc = GRPIC_OK;
    unsigned long long before = 0, after = 0;
    if (FAILS(hipMemcpyAsync(st, x, 3 * n * 8, hipMemcpyHostToDevice, s))) rc = GRPIC_EDEVICE;
    if (!rc && FAILS(hipMemcpyAsync(st + 3 * n, ucov, 3 * n * 8, hipMemcpyHostToDevice, s))) rc = GRPIC_EDEVICE;
    if (!rc && FAILS(hipMemcpyAsync(&before, h->counters + C_LOAD_KEPT, 8, hipMemcpyDeviceToHost, s)))
        rc = GRPIC_EDEVICE;
    // new slots past the last sort's live count: the kernels visit all slots again
    if (!rc && FAILS(hipMemsetAsync(h->counters + C_NALIVE, 0, 8, s))) rc = GRPIC_EDEVICE;
    if (!rc) {
        if (h->mixed)
            launch_load32(h->G, h->h, h->cfg.c, h->cfg.r_rm, st, st + 3 * n, n, species, pp32(h, h->xc, h->uc),
                          h->n_slots, h->counters, s);
        else
            launch_load(h->G, h->h, h->cfg.c, h->cfg.r_rm, st, st + 3 * n, n, species, pp(h, h->xc, h->uc),
                        h->n_slots, h->counters, s);
        rc = check(hipGetLastError());
    }
    if (!rc && FAILS(hipMemcpyAsync(&after, h->counters + C_LOAD_KEPT, 8, hipMemcpyDeviceToHost, s)))
        rc = GRPIC_EDEVICE;
    if (!rc) rc = check(hipStreamSynchronize(s));
    if (rc) return rc;
    h->n_slots += n;
    if (kept) *kept = (int64_t)(after - before);
    return GRPIC_OK;
}
}  // namespace

int grpic_load_particles(grpic_t *h, int32_t species, int64_t n, const double *x, const double *ucov,
                         int64_t *kept) {
    if (!h || n < 0 || (n > 0 && (!x || !ucov))) return GRPIC_EINVAL;
    if (species < 0 || species >= h->cfg.nspecies) return GRPIC_EINVAL;
    if (h->n_slots + n > h->cap) return GRPIC_ENOMEM;
    clear_foreign_error();
    if (kept) *kept = 0;
    if (n == 0) return GRPIC_OK;
    Temp stage(h, (size_t)6 * n * 8);
    if (!stage.p) return GRPIC_ENOMEM;
    return load_staged(h, species, n, x, ucov, kept, (double *)stage.p);
}

int grpic_load_particles_noalloc(grpic_t *h, int32_t species, int64_t n, const double *x, const double *ucov,
                                 int64_t *kept) {
    if (!h || n < 0 || (n > 0 && (!x || !ucov))) return GRPIC_EINVAL;
    if (species < 0 || species >= h->cfg.nspecies) return GRPIC_EINVAL;
    if (n > kNoAllocLoadMax) {
        fprintf(stderr, "grpic: grpic_load_particles_noalloc loads at most %lld particles per call, got %lld\n",
                (long long)kNoAllocLoadMax, (long long)n);
        return GRPIC_EINVAL;
    }
    if (h->n_slots + n > h->cap) return GRPIC_ENOMEM;
    clear_foreign_error();
    if (kept) *kept = 0;
    if (n == 0) return GRPIC_OK;
    if (!h->noalloc_staging) return GRPIC_EDEVICE;
    return load_staged(h, species, n, x, ucov, kept, h->noalloc_staging);
}

int grpic_step(grpic_t *h, int32_t nsteps) {
    clear_foreign_error();
    if (!h || nsteps < 0) return GRPIC_EINVAL;
    if (*h->flags_host & kFlagFixedRange) h->sticky = GRPIC_EOVERFLOW;
    if (h->sticky) return h->sticky;
    for (int i = 0; i < nsteps; i++) {
        int rc = one_step(h);
        if (rc) {
            h->sticky = rc;
            return rc;
        }
    }
    // the flags reach the host asynchronously; a later call reports them
    int rc = check(hipMemcpyAsync((void *)h->flags_host, h->counters + C_FLAGS, 8, hipMemcpyDeviceToHost, h->stream));
    if (rc) h->sticky = rc;
    return rc;
}

int grpic_push_only(grpic_t *h, int32_t nsteps) {
    clear_foreign_error();
    if (!h || nsteps < 0) return GRPIC_EINVAL;
    if (h->mixed)
        launch_node_tensor<float>(h->G, h->h, h->F32, h->stream);
    else
        launch_node_tensor<double>(h->G, h->h, h->F64, h->stream);
    for (int i = 0; i < nsteps; i++) {
        push_particles(h);
        h->xc = 1 - h->xc;
    }
    return check(hipGetLastError());
}

int grpic_particle_count(grpic_t *h, int64_t *n_slots, int64_t *capacity) {
    if (!h) return GRPIC_EINVAL;
    if (n_slots) *n_slots = h->n_slots;
    if (capacity) *capacity = h->cap;
    return GRPIC_OK;
}

int grpic_dump_particles(grpic_t *h, double *x, double *u, uint8_t *sp) {
    if (!h) return GRPIC_EINVAL;
    int64_t n = h->n_slots;
    hipStream_t s = h->stream;
    Temp tmp(h, h->mixed ? (size_t)7 * (n > 0 ? n : 1) * 8 : 8);
    if (!tmp.p) return GRPIC_ENOMEM;
    ParticlePtrs P = f64_view(h, (double *)tmp.p);
    int rc = GRPIC_OK;
    for (int q = 0; q < 3 && x && !rc; q++) rc = check(hipMemcpyAsync(x + q * n, P.x[q], n * 8, hipMemcpyDeviceToHost, s));
    for (int q = 0; q < 4 && u && !rc; q++) rc = check(hipMemcpyAsync(u + q * n, P.u[q], n * 8, hipMemcpyDeviceToHost, s));
    if (sp && !rc) rc = check(hipMemcpyAsync(sp, P.sp, n, hipMemcpyDeviceToHost, s));
    if (!rc) rc = check(hipStreamSynchronize(s));
    return rc;
}

int grpic_restore_particles(grpic_t *h, int64_t n, const double *x, const double *u, const uint8_t *sp) {
    if (!h || n < 0 || n > h->cap || (n > 0 && (!x || !u || !sp))) return GRPIC_EINVAL;
    hipStream_t s = h->stream;
    int rc = GRPIC_OK;
    if (h->mixed) {
        Temp tmp(h, (size_t)7 * (n > 0 ? n : 1) * 8);
        if (!tmp.p) return GRPIC_ENOMEM;
        double *t = (double *)tmp.p;
        rc = check(hipMemcpyAsync(t, x, 3 * n * 8, hipMemcpyHostToDevice, s));
        if (!rc) rc = check(hipMemcpyAsync(t + 3 * n, u, 4 * n * 8, hipMemcpyHostToDevice, s));
        if (!rc) launch_from_f64(t, t + 3 * n, pp32(h, h->xc, h->uc), n, s);
        if (!rc) rc = check(hipStreamSynchronize(s));
    } else {
        for (int q = 0; q < 3 && !rc; q++)
            rc = check(hipMemcpyAsync(h->px[h->xc][q], x + q * n, n * 8, hipMemcpyHostToDevice, s));
        for (int q = 0; q < 4 && !rc; q++)
            rc = check(hipMemcpyAsync(h->pu[h->uc][q], u + q * n, n * 8, hipMemcpyHostToDevice, s));
    }
    if (!rc) rc = check(hipMemcpyAsync(h->psp[h->uc], sp, n, hipMemcpyHostToDevice, s));
    // removed particles may now sit anywhere: the kernels visit all slots
    if (!rc) rc = check(hipMemsetAsync(h->counters + C_NALIVE, 0, 8, s));
    if (!rc) rc = check(hipStreamSynchronize(s));
    if (!rc) h->n_slots = n;
    return rc;
}

int64_t grpic_field_size(const grpic_t *h) { return h ? h->G.gsize() : 0; }

int grpic_dump_fields(grpic_t *h, int32_t which, double *out) {
    if (!h || !out || which < 0 || which > 4) return GRPIC_EINVAL;
    return h->mixed ? dump_fields_t<float>(h, which, out) : dump_fields_t<double>(h, which, out);
}

int grpic_restore_fields(grpic_t *h, const double *D, const double *B) {
    if (!h || !D || !B) return GRPIC_EINVAL;
    return h->mixed ? restore_fields_t<float>(h, D, B) : restore_fields_t<double>(h, D, B);
}

namespace {
// Checkpoint layout (host, 8-byte aligned): StateHeader, then D [3][gs] and
// B [3][gs] as doubles, rho_abs [gs] and the counters [kCounterWords] as
// uint64, then the particles as the run stores them: FP64 runs x [3][n] and
// u [4][n] as doubles; FP32-mixed runs the packed cell [n] as int32, the
// offsets [3][n] and u [4][n] as floats (so a resumed run holds the same bits);
// then sp [n] bytes.
const char kStateMagic[8] = {'G', 'R', 'P', 'I', 'C', 'S', 'T', '2'};
struct StateHeader {
    char magic[8];
    int64_t total_bytes;
    grpic_config key;  // configuration, normalised by state_key
    int64_t n_slots, step_count, field_size, counter_words;
};

// The configuration fields that determine the evolution, in a zeroed struct
// (no padding garbage, no capacity or allocator).
void state_key(const grpic_config *c, grpic_config *k) {
    memset(k, 0, sizeof(*k));
    k->nx = c->nx;
    k->ny = c->ny;
    k->nz = c->nz;
    k->precision = c->precision;
    k->gamma_mode = c->gamma_mode;
    k->deposit_mode = c->deposit_mode;
    k->field_iters = c->field_iters;
    k->sort_every = c->sort_every;
    k->tile = c->tile;
    k->fp_bits = c->fp_bits;
    k->nspecies = c->nspecies;
    k->init_covariant = c->init_covariant;
    k->rk_mode = c->rk_mode;
    k->gather_mode = c->gather_mode;
    k->gather_weights = c->gather_weights;
    k->c = c->c;
    k->dt = c->dt;
    k->m = c->m;
    k->a = c->a;
    for (int i = 0; i < 3; i++) {
        k->center[i] = c->center[i];
        k->B0[i] = c->B0[i];
    }
    k->r_rm = c->r_rm;
    k->r_exc = c->r_exc;
    k->r_damp = c->r_damp;
    k->damp_max = c->damp_max;
    k->outer_layer = c->outer_layer;
    k->outer_damp = c->outer_damp;
    for (int i = 0; i < GRPIC_MAX_SPECIES; i++) {
        k->charge[i] = c->charge[i];
        k->mass[i] = c->mass[i];
    }
}

int64_t state_bytes_for(int64_t gs, int64_t n, bool mixed) {
    int64_t b = (int64_t)sizeof(StateHeader) + 8 * (6 * gs + gs + kCounterWords) + (mixed ? 32 : 56) * n + n;
    return (b + 7) & ~(int64_t)7;
}

// Particle section of a state: copy the stored representation out or in.
int state_particles(grpic_t *h, char *p, int64_t n, bool out) {
    hipStream_t s = h->stream;
    const hipMemcpyKind kind = out ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice;
    std::vector<std::pair<void *, size_t>> parts;  // device pointer, bytes
    if (h->mixed) {
        parts.push_back({h->pcell[h->xc], (size_t)n * 4});
        for (int q = 0; q < 3; q++) parts.push_back({h->poff[h->xc][q], (size_t)n * 4});
        for (int q = 0; q < 4; q++) parts.push_back({h->pu32[h->uc][q], (size_t)n * 4});
    } else {
        for (int q = 0; q < 3; q++) parts.push_back({h->px[h->xc][q], (size_t)n * 8});
        for (int q = 0; q < 4; q++) parts.push_back({h->pu[h->uc][q], (size_t)n * 8});
    }
    parts.push_back({h->psp[h->uc], (size_t)n});
    int rc = GRPIC_OK;
    for (auto &pr : parts) {
        if (!rc && pr.second)
            rc = out ? check(hipMemcpyAsync(p, pr.first, pr.second, kind, s))
                     : check(hipMemcpyAsync(pr.first, p, pr.second, kind, s));
        p += pr.second;
    }
    if (!rc) rc = check(hipStreamSynchronize(s));
    return rc;
}
}  // namespace

int64_t grpic_state_bytes(grpic_t *h) {
    if (!h) return GRPIC_EINVAL;
    return state_bytes_for(h->G.gsize(), h->n_slots, h->mixed);
}

int grpic_save_state(grpic_t *h, void *buf, int64_t bytes) {
    clear_foreign_error();
    if (!h || !buf || ((uintptr_t)buf & 7)) return GRPIC_EINVAL;
    const int64_t gs = h->G.gsize(), n = h->n_slots, total = state_bytes_for(gs, n, h->mixed);
    if (bytes < total) return GRPIC_EINVAL;
    char *b = (char *)buf;
    StateHeader *hd = (StateHeader *)b;
    memcpy(hd->magic, kStateMagic, 8);
    hd->total_bytes = total;
    state_key(&h->cfg, &hd->key);
    hd->n_slots = n;
    hd->step_count = h->step_count;
    hd->field_size = gs;
    hd->counter_words = kCounterWords;
    double *D = (double *)(b + sizeof(StateHeader));
    double *B = D + 3 * gs;
    unsigned long long *rho = (unsigned long long *)(B + 3 * gs);
    unsigned long long *cnt = rho + gs;
    char *parts = (char *)(cnt + kCounterWords);
    int rc = grpic_dump_fields(h, 0, D);
    if (!rc) rc = grpic_dump_fields(h, 1, B);
    hipStream_t s = h->stream;
    unsigned long long *rho_dev = h->mixed ? h->F32.rho_abs : h->F64.rho_abs;
    if (!rc) rc = check(hipMemcpyAsync(rho, rho_dev, gs * 8, hipMemcpyDeviceToHost, s));
    if (!rc) rc = check(hipMemcpyAsync(cnt, h->counters, kCounterWords * 8, hipMemcpyDeviceToHost, s));
    if (!rc) rc = check(hipStreamSynchronize(s));
    if (!rc && n > 0) rc = state_particles(h, parts, n, true);
    return rc;
}

int grpic_load_state(grpic_t *h, const void *buf, int64_t bytes) {
    clear_foreign_error();
    if (!h || !buf || ((uintptr_t)buf & 7) || bytes < (int64_t)sizeof(StateHeader)) return GRPIC_EINVAL;
    const char *b = (const char *)buf;
    const StateHeader *hd = (const StateHeader *)b;
    grpic_config key;
    state_key(&h->cfg, &key);
    const int64_t gs = h->G.gsize();
    if (memcmp(hd->magic, kStateMagic, 8) || memcmp(&hd->key, &key, sizeof(key)) || hd->field_size != gs ||
        hd->counter_words != kCounterWords || hd->n_slots < 0 || hd->n_slots > h->cap || hd->step_count < 0 ||
        hd->total_bytes != state_bytes_for(gs, hd->n_slots, h->mixed) || bytes < hd->total_bytes)
        return GRPIC_EINVAL;
    const int64_t n = hd->n_slots;
    const double *D = (const double *)(b + sizeof(StateHeader));
    const double *B = D + 3 * gs;
    const unsigned long long *rho = (const unsigned long long *)(B + 3 * gs);
    const unsigned long long *cnt = rho + gs;
    char *parts = (char *)(cnt + kCounterWords);
    int rc = grpic_restore_fields(h, D, B);
    hipStream_t s = h->stream;
    unsigned long long *rho_dev = h->mixed ? h->F32.rho_abs : h->F64.rho_abs;
    if (!rc) rc = check(hipMemcpyAsync(rho_dev, rho, gs * 8, hipMemcpyHostToDevice, s));
    if (!rc) rc = check(hipMemcpyAsync(h->counters, cnt, kCounterWords * 8, hipMemcpyHostToDevice, s));
    if (!rc) rc = check(hipStreamSynchronize(s));
    if (!rc) rc = state_particles(h, parts, n, false);
    if (!rc) {
        h->n_slots = n;
        h->step_count = hd->step_count;
    }
    return rc;
}

int grpic_dump_nodes(grpic_t *h, double *out) {
    if (!h || !out) return GRPIC_EINVAL;
    int64_t cnt = h->G.nnodes() * 16;
    return h->mixed ? copy_field_out<float>(h, h->F32.node, out, cnt) : copy_field_out<double>(h, h->F64.node, out, cnt);
}

int grpic_sort(grpic_t *h, uint32_t *keys_out, int64_t *perm_out) {
    clear_foreign_error();
    if (!h) return GRPIC_EINVAL;
    int64_t n = h->n_slots;
    uint32_t *fk = nullptr, *fi = nullptr;
    int rc = do_sort(h, true, &fk, &fi);
    if (rc) return rc;
    if (n == 0) return GRPIC_OK;
    hipStream_t s = h->stream;
    const bool out = keys_out || perm_out;
    std::vector<uint32_t> k(out ? n : 0), p(out ? n : 0);
    unsigned long long cnt[C_NCOUNTERS];
    rc = out ? check(hipMemcpyAsync(k.data(), fk, n * 4, hipMemcpyDeviceToHost, s)) : GRPIC_OK;
    if (!rc && out) rc = check(hipMemcpyAsync(p.data(), fi, n * 4, hipMemcpyDeviceToHost, s));
    if (!rc) rc = check(hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    if (!rc) rc = check(hipStreamSynchronize(s));
    if (rc) return rc;
    uint32_t sentinel = h->key_bits >= 32 ? 0xFFFFFFFFu : ((1u << h->key_bits) - 1u);
    for (int64_t i = 0; out && i < n; i++) {
        if (keys_out) keys_out[i] = k[i] == sentinel ? 0xFFFFFFFFu : k[i];
        if (perm_out) perm_out[i] = (int64_t)p[i];
    }
    if (n > 0) h->n_slots = (int64_t)cnt[C_NALIVE];
    return GRPIC_OK;
}

int grpic_diagnostics(grpic_t *h, grpic_diag *out) {
    clear_foreign_error();
    if (!h || !out) return GRPIC_EINVAL;
    memset(out, 0, sizeof(*out));
    hipStream_t s = h->stream;
    int64_t n = h->n_slots;
    Temp tmp(h, h->mixed ? (size_t)7 * (n > 0 ? n : 1) * 8 : 8);
    if (!tmp.p) return GRPIC_ENOMEM;
    ParticlePtrs P = f64_view(h, (double *)tmp.p);
    DiagOut d;
    int rc;
    // derived fields of the current state (frozen points keep their initial values)
    if (h->mixed) {
        launch_derived<float>(h->G, h->h, h->F32, true, true, true, s);
        rc = run_diag<float>(h->G, h->h, h->cfg.c, h->rscale, h->S, P, n, h->F32, h->cfg.r_damp, h->cfg.damp_max,
                             h->cfg.outer_layer, h->cfg.outer_damp, h->rho_scratch, h->red, h->red_cap, d, s);
    } else {
        launch_derived<double>(h->G, h->h, h->F64, true, true, true, s);
        rc = run_diag<double>(h->G, h->h, h->cfg.c, h->rscale, h->S, P, n, h->F64, h->cfg.r_damp, h->cfg.damp_max,
                              h->cfg.outer_layer, h->cfg.outer_damp, h->rho_scratch, h->red, h->red_cap, d, s);
    }
    if (rc) return GRPIC_EDEVICE;
    std::vector<unsigned long long> cnt(kCounterWords);
    rc = check(hipMemcpyAsync(cnt.data(), h->counters, kCounterWords * 8, hipMemcpyDeviceToHost, s));
    if (!rc) rc = check(hipStreamSynchronize(s));
    if (rc) return rc;
    for (int q = 0; q < GRPIC_MAX_SPECIES; q++) out->n_alive[q] = d.n_alive[q];
    out->n_removed_horizon = (int64_t)cnt[C_REMOVED_HORIZON];
    out->n_removed_outer = (int64_t)cnt[C_REMOVED_OUTER];
    out->gamma_clamps = (int64_t)cnt[C_GAMMA_CLAMPS];
    out->flags = (int64_t)cnt[C_FLAGS];
    out->charge_total = d.charge_total;
    out->energy_particles = d.energy_particles;
    out->lz_particles = d.lz_particles;
    out->energy_field = d.energy_field;
    out->gauss_residual_max = d.gauss_max;
    out->mass_shell_residual_max = d.shell_max;
    out->deposit_blocks_lds = (int64_t)cnt[C_DEP_LDS];
    out->deposit_blocks_global = (int64_t)cnt[C_DEP_GLOBAL];
    for (int q = 0; q < kPushedSlots; q++) {
        out->push_blocks_lds += (int64_t)cnt[pushed_index((unsigned)q) + kPushedLds];
        out->push_blocks_global += (int64_t)cnt[pushed_index((unsigned)q) + kPushedGlobal];
    }
    if ((cnt[C_FLAGS] & kFlagFixedRange) && !h->sticky) h->sticky = GRPIC_EOVERFLOW;
    return h->sticky ? h->sticky : GRPIC_OK;
}

int grpic_set_timing(grpic_t *h, int32_t enable) {
    if (!h) return GRPIC_EINVAL;
    h->timing = enable ? 1 : 0;
    return GRPIC_OK;
}

int grpic_set_graphs(grpic_t *h, int32_t enable) {
    if (!h) return GRPIC_EINVAL;
    h->use_graphs = enable ? 1 : 0;
    if (!h->use_graphs) {
        int rc = check(hipStreamSynchronize(h->stream));
        drop_cycle_graphs(h);
        return rc;
    }
    return GRPIC_OK;
}

int grpic_read_timing(grpic_t *h, double *ms, int64_t *launches) {
    if (!h) return GRPIC_EINVAL;
    int rc = check(hipStreamSynchronize(h->stream));
    for (int t = 0; t < GRPIC_NTIMERS; t++) {
        double tot = 0.0;
        for (auto &pr : h->ev_used[t]) {
            float e = 0.0f;
            if (!rc) rc = check(hipEventElapsedTime(&e, pr.first, pr.second));
            tot += e;
            h->ev_pool.push_back(pr.first);
            h->ev_pool.push_back(pr.second);
        }
        if (ms) ms[t] = tot;
        if (launches) launches[t] = (int64_t)h->ev_used[t].size();
        h->ev_used[t].clear();
    }
    return rc;
}

int grpic_particle_steps(grpic_t *h, int64_t *out) {
    if (!h || !out) return GRPIC_EINVAL;
    std::vector<unsigned long long> v(kCounterWords);
    int rc = check(hipMemcpyAsync(v.data(), h->counters, kCounterWords * 8, hipMemcpyDeviceToHost, h->stream));
    if (!rc) rc = check(hipStreamSynchronize(h->stream));
    unsigned long long sum = 0;
    for (int s = 0; s < kPushedSlots; s++) sum += v[pushed_index((unsigned)s)];
    *out = (int64_t)sum;
    return rc;
}

}  // extern "C"
