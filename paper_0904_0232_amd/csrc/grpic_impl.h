// Internal state shared by the kernel files and the C ABI implementation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grpic_dev.h"

namespace grpic {

// Device pointers of the field state, stored in T (double for the FP64
// form, float for the FP32-mixed form).  Every array of a staggered
// component has Grid::gsize() entries; node arrays have Grid::nnodes().
template <typename T>
struct FieldPtrsT {
    T *D[3], *B[3];         // evolved: F^{c4} at E points, covariant pairs at B points
    T *E[3], *H[3];         // derived: F_{c4} at E points, contravariant pairs at B points
    T *D0[3], *B0[3];       // initial evolved values (frozen points, relaxation target)
    T *E0[3], *H0[3];       // initial derived values (frozen points)
    T *Dsave[3], *Bsave[3]; // D^n and B^{n-1/2} during the fixed-point passes
    unsigned long long *Jint[3];  // int64 fixed-point current on E points
    unsigned long long *rho_abs;  // int64 fixed-point charge removed at the horizon (nodes, ghosted)
    uint8_t *mask;          // update bits per ghosted index
    T *w;                   // [6][nnodes] scratch (S - I) P v
    T *node;                // [nnodes][16] mixed tensor F^a_b
};
using FieldPtrs = FieldPtrsT<double>;

// FP32-mixed particle storage: packed cell (i+1) | (j+1) << 10 | (k+1) << 20,
// FP32 offset inside the cell, FP32 contravariant four-velocity.
struct ParticlePtrs32 {
    int32_t *cell;
    float *off[3];
    float *u[4];
    uint8_t *sp;
};

__host__ __device__ inline int32_t pack_cell(int i, int j, int k) {
    return (int32_t)((uint32_t)(i + 1) | ((uint32_t)(j + 1) << 10) | ((uint32_t)(k + 1) << 20));
}
__host__ __device__ inline void unpack_cell(int32_t c, int &i, int &j, int &k) {
    uint32_t u = (uint32_t)c;
    i = (int)(u & 1023u) - 1;
    j = (int)((u >> 10) & 1023u) - 1;
    k = (int)((u >> 20) & 1023u) - 1;
}

// FP64 particle storage (SoA), two buffers for the sort and for x_n/x_{n+1}.
struct ParticlePtrs {
    double *x[3];
    double *u[4];
    uint8_t *sp;
};

struct Species {
    double qm[kMaxSpecies];
    double charge[kMaxSpecies];
    double mass[kMaxSpecies];
};

// Distance of a point (node coordinates) from the nearest outer face.
__device__ __forceinline__ double outer_distance(const Grid &G, double X, double Y, double Z) {
    double d = fmin(X, (double)G.nx - X);
    d = fmin(d, fmin(Y, (double)G.ny - Y));
    return fmin(d, fmin(Z, (double)G.nz - Z));
}

// Device counters, one 64-bit word each.
enum Counter {
    C_NALIVE = 0,      // live slots after the last cell sort (0: none since the slots last changed)
    C_GAMMA_CLAMPS = 1,
    C_REMOVED_HORIZON = 2,
    C_REMOVED_OUTER = 3,
    C_FLAGS = 4,
    C_LOAD_KEPT = 5,
    C_DEP_LDS = 6,     // deposit blocks that summed their current in an LDS box
    C_DEP_GLOBAL = 7,  // deposit blocks that added it with global atomics
    C_NCOUNTERS = 8
};

// Slots the particle kernels need to visit: the cell sort moves removed
// particles to the end and leaves the live count in C_NALIVE, and later
// removals only mark slots in place, so every slot from there on holds a
// removed particle.  Loading or restoring particles resets the count to 0,
// which means all n slots.
__device__ __forceinline__ int64_t live_bound(const unsigned long long *counters, int64_t n) {
    const unsigned long long a = counters[C_NALIVE];
    return (a > 0 && (int64_t)a < n) ? (int64_t)a : n;
}

// Bits of C_FLAGS (sticky).
constexpr unsigned long long kFlagLongMove = 1ull;    // a move longer than a cell (not deposited)
constexpr unsigned long long kFlagFixedRange = 2ull;  // an int64 fixed-point sum left the int64 range

// Add v to an int64 fixed-point sum in device memory.  When the partial sum
// leaves the int64 range (old and v of one sign, the result of the other)
// flags bit kFlagFixedRange is raised.  A sum whose partial sums never wrap,
// in the order the atomics happened, is exact; a flagged sum may be wrong.
__device__ __forceinline__ bool fixed_wrapped(long long old, long long v) {
    const long long res = (long long)((unsigned long long)old + (unsigned long long)v);
    return ((old ^ res) & (v ^ res)) < 0;
}
__device__ __forceinline__ void fixed_add_checked(unsigned long long *p, long long v, unsigned long long *flags) {
    const long long old = (long long)atomicAdd(p, (unsigned long long)v);
    if (fixed_wrapped(old, v)) atomicOr(flags, kFlagFixedRange);
}

// Flush of a block's LDS current box (3 V int64 sums, edge direction
// major, then z, y, x within the box at blo) into the global sums.  The box
// sums themselves cannot wrap: a deposit block holds at most 1024
// particles, each adding less than 2^(fp_bits + 1) <= 2^51 to an edge.  The
// global additions return the old value for the range check, four per thread
// in flight before their results are examined.
__device__ __forceinline__ void flush_box(const unsigned long long *sm, int V, int bx, int by, const int blo[3],
                                          unsigned long long *const J[3], const Grid &G, unsigned long long *flags) {
    const float inv_bx = __builtin_amdgcn_rcpf((float)bx), inv_bxy = __builtin_amdgcn_rcpf((float)(bx * by));
    bool wrapped = false;
    for (int e0 = threadIdx.x; e0 < 3 * V; e0 += 4 * (int)blockDim.x) {
        long long v[4], old[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int e = e0 + q * (int)blockDim.x;
            v[q] = e < 3 * V ? (long long)sm[e] : 0ll;
            old[q] = 0;
            if (v[q] != 0) {
                const int K = e >= 2 * V ? 2 : (e >= V ? 1 : 0), l = e - K * V;
                const int lk = small_div(l, inv_bxy), r = l - lk * bx * by, lj = small_div(r, inv_bx),
                          li = r - lj * bx;
                old[q] = (long long)atomicAdd(&J[K][G.g(blo[0] + li, blo[1] + lj, blo[2] + lk)],
                                              (unsigned long long)v[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; q++) wrapped |= fixed_wrapped(old[q], v[q]);
    }
    if (wrapped) atomicOr(flags, kFlagFixedRange);
}

// The particle-step counter (live particles pushed, summed over steps) gets
// one increment per wave of every push: it is spread over kPushedSlots cache
// lines after the first, so same-address atomics do not serialise the push.
// The counter is the sum of the slots.  The next two words of each slot
// count push blocks with live particles that staged an LDS node box
// (kPushedLds) and that did not (kPushedGlobal), once per block.
constexpr int kPushedSlots = 64;
constexpr int kCounterWords = 16 * (1 + kPushedSlots);
constexpr int kPushedLds = 1, kPushedGlobal = 2;
__host__ __device__ inline int pushed_index(unsigned block) { return 16 * (1 + (int)(block & (kPushedSlots - 1))); }

struct PushParams {
    Grid G;
    Hole h;
    double c, dt;
    double inv_c;        // 1 / c
    double dt_2c;        // dt / (2 c)
    double dt_6;         // dt / 6
    int gamma_mode;
    int rk_mode;      // GRPIC_RK_* (FP64 pusher only)
    int gather_mode;  // GRPIC_GATHER_* (FP64 pusher only)
    int gather_weights;  // GRPIC_WEIGHTS_* (FP64 pusher only)
    int64_t n;  // slots to process
};

// field kernels (T = double or float)
template <typename T> void launch_bake(const Grid &G, const Hole &h, FieldPtrsT<T> &F, hipStream_t s);
template <typename T>
void launch_init_fields(const Grid &G, const Hole &h, FieldPtrsT<T> &F, const double B0[3], int covariant,
                        hipStream_t s);
template <typename T>
void launch_derived(const Grid &G, const Hole &h, FieldPtrsT<T> &F, bool use_ref, bool do_e, bool do_h,
                    hipStream_t s);
template <typename T>
void launch_bhalf(const Grid &G, FieldPtrsT<T> &F, const T *const Bin[3], double hstep, hipStream_t s);
template <typename T>
void launch_dstep(const Grid &G, FieldPtrsT<T> &F, const T *const Din[3], double dx4, double fpc,
                  double inv_jscale, hipStream_t s);
template <typename T>
void launch_relax(const Grid &G, const Hole &h, FieldPtrsT<T> &F, double r_damp, double damp_max, hipStream_t s);
// Outer absorbing layer: updated points closer than L to the nearest face
// relax toward their initial values by damp ((L - d)/L)^2.
template <typename T>
void launch_relax_outer(const Grid &G, FieldPtrsT<T> &F, double L, double damp, hipStream_t s);
template <typename T> void launch_node_tensor(const Grid &G, const Hole &h, FieldPtrsT<T> &F, hipStream_t s);
// Bsave <- B (which = 0) or Dsave <- D (which = 1), all three components.
template <typename T> void launch_save(const Grid &G, FieldPtrsT<T> &F, int which, hipStream_t s);
// Clear the three int64 current arrays.
void launch_zero3_u64(unsigned long long *const p[3], int64_t n, hipStream_t s);

// particle kernels
void launch_push(const PushParams &P, const Species &S, const double *node, ParticlePtrs in, ParticlePtrs out,
                 unsigned long long *counters, hipStream_t s);
void launch_deposit(const Grid &G, const Hole &h, double dt, int deposit_mode, double r_rm, double jscale,
                    double rscale, const Species &S, ParticlePtrs xold, ParticlePtrs xnew, int64_t n,
                    FieldPtrs &F, unsigned long long *counters, hipStream_t s);
void launch_load(const Grid &G, const Hole &h, double c, double r_rm, const double *xin, const double *ucin,
                 int64_t n, int species, ParticlePtrs out, int64_t offset, unsigned long long *counters,
                 hipStream_t s);
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s);

// FP32-mixed particle kernels
struct Mixed {
    double r_fp64;  // metric and Christoffel symbols in FP64 when r < r_fp64
};
void launch_push32(const PushParams &P, const Mixed &M, const Species &S, const float *node, ParticlePtrs32 in,
                   ParticlePtrs32 out, unsigned long long *counters, hipStream_t s);
void launch_deposit32(const Grid &G, const Hole &h, const Mixed &M, double dt, int deposit_mode, double r_rm,
                      double jscale, double rscale, const Species &S, ParticlePtrs32 xold, ParticlePtrs32 xnew,
                      int64_t n, FieldPtrsT<float> &F, unsigned long long *counters, hipStream_t s);
struct Dep32 {
    Grid G;
    Hole h;
    double r_fp64;
    float r_fp64_sq;  // r_fp64^2: FP32 densities only beyond it
    float af, m2;     // a and 2 m in FP32
    float inv_dt;
    double jscale;
    int curved;
};
void launch_load32(const Grid &G, const Hole &h, double c, double r_rm, const double *xin, const double *ucin,
                   int64_t n, int species, ParticlePtrs32 out, int64_t offset, unsigned long long *counters,
                   hipStream_t s);
void launch_to_f64(ParticlePtrs32 in, double *x, double *u, int64_t n, hipStream_t s);
void launch_from_f64(const double *x, const double *u, ParticlePtrs32 out, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// Serving batch (FP32-mixed form): one launch per cycle stage covers every
// active run.  The launches are persistent: a fixed grid whose blocks walk
// the logical blocks of all runs, each run owning a contiguous range of
// logical blocks per kind of work, so a logical block belongs to one run.
// The run table lives in device memory and is rewritten before every
// iteration, so a captured iteration replays unchanged while runs come and
// go and their buffers swap.
enum BatchKind { BK_NODE = 0, BK_GRID, BK_RELAX, BK_PUSH, BK_DEP, BK_SORT_SLOT, BK_SORT_TILE, BK_SORT_SCAN,
                 BK_NKINDS };
constexpr int kBatchBlock = 256;     // threads per block of the field kinds
constexpr int kMaxBatchRuns = 64;

constexpr int kSortMaxPasses = 4;  // digits of at most 9 bits cover 32-bit keys

// One run's cell sort inside a batched iteration (n = 0: no sort is due):
// the pass plan and, per pass, the key and value arrays read and written
// (the same ping-pong as a single run's sort).
struct BatchSort {
    int64_t n;        // slots
    int64_t ntiles;   // tiles of the radix passes
    int64_t nchunks;  // scan chunks of the widest pass
    int tile, nTx, nTy;
    uint32_t sentinel;
    int passes;
    int shift[kSortMaxPasses], bits[kSortMaxPasses];
    uint32_t *kin[kSortMaxPasses], *vin[kSortMaxPasses], *kout[kSortMaxPasses], *vout[kSortMaxPasses];
    uint32_t *counts, *sums;
    const uint32_t *final_idx;
    ParticlePtrs32 in, out;
};

struct BatchRun32 {
    int64_t off[BK_NKINDS];  // first logical block of this run per kind
    Grid G;
    Hole h;
    FieldPtrsT<float> F;
    float hstep;             // c dt / 2
    double c, dt;
    float fpc;               // 4 pi / c
    double inv_jscale;
    int field_iters;
    int relax_box[6];        // i0, j0, k0, bx, by, bz (bx = 0: no relaxation)
    double r_damp, damp_max;
    PushParams P;            // P.n = particle slots
    Mixed M;
    Species S;
    ParticlePtrs32 cur, nxt;  // state at time n and the buffers of time n+1
    unsigned long long *counters;
    Dep32 D;
    double r_rm, rscale;
    BatchSort sort;
};

struct BatchTable {
    int nruns;
    int64_t total[BK_NKINDS];  // logical blocks per kind over all runs
    BatchRun32 run[kMaxBatchRuns];
};

// Stage identifiers of the batched field launches.
enum BatchFieldOp { BF_SAVE_B, BF_NODE_W, BF_ECOV, BF_BHALF_SAVED, BF_NODE_TENSOR, BF_BHALF_CUR, BF_ZERO_J,
                    BF_SAVE_D, BF_HFIELD, BF_DSTEP, BF_RELAX };
// The run owning logical block lb of a kind: the last run whose first block
// is <= lb (runs are stored in increasing block order).
__device__ __forceinline__ int batch_run_of(const BatchTable *__restrict__ T, int kind, int64_t lb) {
    int lo = 0, hi = T->nruns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T->run[mid].off[kind] <= lb)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}
Dep32 make_dep32(const Grid &G, const Hole &h, const Mixed &M, double dt, int deposit_mode, double jscale);
void launch_batch_field(int op, const BatchTable *table, int it, int grid, hipStream_t s);
void launch_batch_push32(const BatchTable *table, int grid, hipStream_t s);
void launch_batch_deposit32(const BatchTable *table, int grid, hipStream_t s);
// logical blocks of one run per kind (field kinds in kBatchBlock threads)
int64_t batch_blocks(int kind, const Grid &G, const int relax_box[6], int64_t n_slots);
void relax_box_of(const Grid &G, const Hole &h, double r_damp, double damp_max, int box[6]);

// sort
// Scratch bytes of the sort for up to `capacity` slots (digit counts per
// tile and the scan's chunk sums).
size_t sort_temp_bytes(int64_t capacity);
// Stable sort of the n slots by tile-major cell key into `out`, removed
// particles last; counters[C_NALIVE] receives the live count.  keys, keys_alt,
// idx and idx_alt (n entries each) carry the keys and slot indices between
// passes.  keep: *final_keys and *final_idx point at the sorted keys and the
// original slot of each sorted position (else NULL).
void launch_sort(const Grid &G, int tile, int64_t n, ParticlePtrs in, ParticlePtrs out, uint32_t *keys,
                 uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, int key_bits, bool keep,
                 uint32_t **final_keys, uint32_t **final_idx, unsigned long long *counters, hipStream_t s);
void launch_sort32(const Grid &G, int tile, int64_t n, ParticlePtrs32 in, ParticlePtrs32 out, uint32_t *keys,
                   uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, int key_bits, bool keep,
                   uint32_t **final_keys, uint32_t **final_idx, unsigned long long *counters, hipStream_t s);
// The batched form of launch_sort32: J describes the sort of one run (the
// same arguments), and the batched launches sort every run of the table
// whose J.n > 0, up to `passes` radix passes (the most any of them needs).
void batch_sort_job(const Grid &G, int tile, int64_t n, ParticlePtrs32 in, ParticlePtrs32 out, uint32_t *keys,
                    uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, int key_bits, BatchSort &J);
// logical blocks of a run's sort per kind (BK_SORT_*)
int64_t batch_sort_blocks(int kind, const BatchSort &J);
void launch_batch_sort(const BatchTable *table, int passes, hipStream_t s);

// diagnostics: fills host-side partial sums (see diag.hip)
struct DiagOut {
    int64_t n_alive[kMaxSpecies];
    double charge_total, energy_particles, lz_particles, energy_field, gauss_max, shell_max;
};
// P: FP64 particle view (the FP32-mixed form is widened into scratch first)
template <typename T>
int run_diag(const Grid &G, const Hole &h, double c, double rscale, const Species &S, ParticlePtrs P, int64_t n,
             FieldPtrsT<T> &F, double r_damp, double damp_max, double outer_layer, double outer_damp,
             unsigned long long *rho_scratch, double *red_scratch, int64_t red_cap, DiagOut &out, hipStream_t s);

}  // namespace grpic
