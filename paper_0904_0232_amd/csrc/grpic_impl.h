// Internal state shared by the kernel files and the C ABI implementation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grpic_dev.h"

namespace grpic {

// Device pointers of the field state (FP64).  Every array of a staggered
// component has Grid::gsize() entries; node arrays have Grid::nnodes().
struct FieldPtrs {
    double *D[3], *B[3];    // evolved: F^{c4} at E points, covariant pairs at B points
    double *E[3], *H[3];    // derived: F_{c4} at E points, contravariant pairs at B points
    double *D0[3], *B0[3];  // initial evolved values (frozen points, relaxation target)
    double *E0[3], *H0[3];  // initial derived values (frozen points)
    double *Dsave[3], *Bsave[3];  // D^n and B^{n-1/2} during the fixed-point passes
    unsigned long long *Jint[3];  // int64 fixed-point current on E points
    unsigned long long *rho_abs;  // int64 fixed-point charge removed at the horizon (nodes, ghosted)
    uint8_t *mask;          // update bits per ghosted index
    double *dS;             // [21][nnodes] packed S - I
    double *gn;             // [10][nnodes] packed g_ab
    double *w;              // [6][nnodes] scratch (S - I) P v
    double *node;           // [nnodes][16] mixed tensor F^a_b
};

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

// Device counters, one 64-bit word each.
enum Counter {
    C_NALIVE = 0,      // live slots after the last compaction (unused while 0)
    C_GAMMA_CLAMPS = 1,
    C_REMOVED_HORIZON = 2,
    C_REMOVED_OUTER = 3,
    C_FLAGS = 4,
    C_LOAD_KEPT = 5,
    C_PUSHED = 6,      // live particles pushed, summed over steps
    C_NCOUNTERS = 8
};

struct PushParams {
    Grid G;
    Hole h;
    double c, dt;
    int gamma_mode;
    int64_t n;  // slots to process
};

// field kernels
void launch_bake(const Grid &G, const Hole &h, FieldPtrs &F, hipStream_t s);
void launch_init_fields(const Grid &G, const Hole &h, FieldPtrs &F, const double B0[3], int covariant,
                        hipStream_t s);
void launch_derived(const Grid &G, FieldPtrs &F, bool use_ref, bool do_e, bool do_h, hipStream_t s);
void launch_bhalf(const Grid &G, FieldPtrs &F, const double *const Bin[3], double hstep, hipStream_t s);
void launch_dstep(const Grid &G, FieldPtrs &F, const double *const Din[3], double dx4, double fpc,
                  double inv_jscale, hipStream_t s);
void launch_relax(const Grid &G, const Hole &h, FieldPtrs &F, double r_damp, double damp_max, hipStream_t s);
void launch_node_tensor(const Grid &G, FieldPtrs &F, hipStream_t s);

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

// sort
size_t sort_temp_bytes(int64_t capacity);
void launch_sort(const Grid &G, int tile, int64_t n, ParticlePtrs in, ParticlePtrs out, uint32_t *keys,
                 uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, size_t temp_bytes,
                 int key_bits, unsigned long long *counters, hipStream_t s);

// diagnostics: fills host-side partial sums (see diag.hip)
struct DiagOut {
    int64_t n_alive[kMaxSpecies];
    double charge_total, energy_particles, lz_particles, energy_field, gauss_max, shell_max;
};
int run_diag(const Grid &G, const Hole &h, double c, double rscale, const Species &S, ParticlePtrs P, int64_t n,
             FieldPtrs &F, double r_damp, double damp_max, unsigned long long *rho_scratch, double *red_scratch,
             int64_t red_cap, DiagOut &out, hipStream_t s);

}  // namespace grpic
