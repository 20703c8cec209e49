// Device-side data layout and small device helpers shared by the UGKWP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ugkwp {

// device error bits, reported through ugkwp_step_stats.error_word
enum : uint32_t {
    kErrNonPhys = 1u,    // rho <= 0, T <= 0 or non-finite in a cell
    kErrCapacity = 2u,   // particles would exceed the capacity
    kErrLost = 4u,       // a particle exceeded max_crossings
    kErrCellCount = 8u,  // more than 2^20 particles sampled in one cell (particle-id field)
};

enum : int { kTagTF = 1, kTagPos = 2, kTagVel = 3, kTagWall = 4, kTagInject = 5, kTagInt = 6, kTagWallInt = 7,
             kTagGP = 8 };

// internal degrees of freedom supported: gamma = (K + 5)/(K + 3), 0 <= K <= kMaxK
constexpr int kMaxK = 8;

// bucket key flag: the particle flew collisionless for the whole step without meeting a face
// (so it ends in the cell it started in, at x + u dt; its record is not rewritten)
constexpr int32_t kStayBit = 1 << 30;

// the neighbour's local face of a slot whose face is periodic: the neighbour's local face lf2
// and the face's boundary condition b (whose shift a crossing particle takes) as
// lf2 + kPeriodicEntry (b + 1); plain neighbours have entries below kPeriodicEntry
constexpr int32_t kPeriodicEntry = 8;

struct DevBC {
    int32_t type;
    int32_t pad;
    double Tw;
    double Uw[3];
    double Winf[5];
    double shift[3];  // periodic: a particle crossing a face of this condition goes on at x + shift
};

// Parameters of one instance of a batch (constant after set-up).  An instance owns a
// contiguous range of cells and of far-field faces of the concatenated mesh.
struct InstP {
    double mu_ref, omega, cfl, c2;
    int32_t n_ref, n_min, max_cross, recon;  // recon: 0 first order, 1 LSQ + BJ, 2 LSQ + Venkatakrishnan
    double venkat_k;
    unsigned long long seed;
    int32_t cell0, cell1;  // cells [cell0, cell1)
    int32_t ff0, ff1;      // far-field faces [ff0, ff1)
    int32_t sampling;      // hydro-particle velocities: 0 U +- sqrt(T) X (Sec. 2.4(b)), 1 energy-exact,
                           // 2 first-order g_p, 3 independent draws from the equilibrium
    int32_t gks_steps;     // steps n < gks_steps of the instance are wave-only (no particles)
    long long bf0;         // its first input boundary face in the concatenated list
    double pr;             // Prandtl number: 1 the BGK model, otherwise the Shakhov model
};

// Step state of one instance: its own time step, time and step counter, and the counts of
// its last step.
struct InstS {
    unsigned long long dtmin_bits;  // bit pattern of min Omega/Lambda over its cells
    double dt, t;
    long long step;
    long long n_alive, n_sampled, n_injected, n_collided, n_escaped;
    long long moved_total;
    // time averaging: sum of dt over the averaged steps, their number, and the relative change
    // of the average in the last of them
    double avg_D;
    long long avg_n;
    double avg_res;
};

// Step scalars of the whole batch, resident in device memory: the host never reads them
// inside a step.  dt, t and step mirror instance 0.
// wall queue: segment s takes the particles stopped at diffuse walls by the transport
// blocks b with b % kWallSeg == s (one counter per segment, not one for the whole grid);
// a segment holds ceil(blocks / kWallSeg) x (particles per block) entries, so the segments
// need at most kWallSlack entries beyond the capacity
// blocks per instance of the averaging kernel (each a contiguous run of its cells)
constexpr int kAvgBlocks = 64;

constexpr int kWallSeg = 64;
constexpr long long kWallSlack = (long long)kWallSeg * 1024;

struct Scalars {
    unsigned long long dtmin_bits;  // bit pattern of min Omega/Lambda (positive doubles order as integers)
    double dt;
    double t;
    long long step;
    long long n_old;      // particles at the start of the step (grouped by cell)
    long long n_new;      // particles sampled in the step (0 if the capacity check failed)
    long long n_inj;      // free-stream particles entering in the step, stored after the sampled ones
    long long n_alive;    // particles after the step
    unsigned long long n_sampled, n_injected, n_collided, n_escaped, n_cross, n_wall;
    unsigned long long moved_total;  // particles streamed since the state was set
    unsigned int err;
    unsigned int max_cross;  // the most face crossings of one particle in the step
    unsigned int n_big;      // cells with more than 64 new particles this step (k_sample_big's list)
    unsigned int pad;
};

// One particle: position, velocity, mass and id in a 64-byte record, so that a particle
// read from anywhere costs one memory transaction; the cell index lives in its own array.
struct alignas(64) PRec {
    double x[3];
    double u[3];
    double m;
    uint64_t uid;
};

// FP32 form: position and velocity in single precision with the id in a 32-byte record; the
// mass (single precision) in its own array, since transport never reads it.
struct alignas(32) PRec32 {
    float x[3];
    float u[3];
    uint64_t uid;
};

struct Particles {
    PRec *rec;      // FP64 form
    PRec32 *rec32;  // FP32 form
    float *m32;     // FP32 form
    int32_t *cell;
    double *e64;    // internal energy variable |xi|^2 of each particle (K > 0; FP64 form)
    float *e32;     // the same in the FP32 form
};

struct Dev {
    // mesh
    int32_t nc, nf, nbc, pad0;
    const double *vol;      // [nc]
    const double *dS;       // [3][nc]
    const double *orig;     // [3][nc]
    const double *edge;     // [9][nc]  edge k component d at [3k+d][nc]
    const uint8_t *nfc;     // [nc]
    const uint8_t *ctype;   // [nc]
    const double *box;      // [nc][6] lo[3], hi[3] of box hexes (unused for tetrahedra)
    const double4 *plane;   // [nc*6]  (n, d) outward
    const float *box32;     // FP32 copies for the FP32 form
    const float4 *plane32;
    const double *nfar;     // [nc*6] conforming boxes (all_box): the bound of the neighbour across
                            // the face on the far side along the face's axis
    const float *nfar32;    // the same for the FP32 form
    const int2 *nbl;        // [nc*6]  (neighbour or -1-bc, local face in neighbour)
    const int32_t *cface;   // [nc*6]  +-(f+1)
    const int32_t *fown;    // [nf]
    const int32_t *fnb;     // [nf]
    const double *fn;       // [3][nf]
    const double *farea;    // [nf]
    const DevBC *bc;        // [nbc]
    const double *xc;       // [3][nc] cell centres (second order)
    const double *lfx;      // [nc*6][3] local face centres (second order)
    const double *fx;       // [3][nf] face centres (second order)
    int32_t nff, pad1;      // far-field faces
    const int4 *ffi;        // [nff]  (cell, local face | triangle << 8, input boundary-face index, bc)
    const double *ffg;      // [nff][10]  corner, two edges, area of the face as listed
    const uint8_t *bflf;    // [n_bfaces]  local face of an input boundary face
    // parameters
    int32_t n_inst, prec;   // prec: 0 FP64 plain, 1 FP32 form
    int32_t K;              // internal degrees of freedom of the gas (every instance)
    int32_t gp_any;         // some instance draws its hydro particles one by one (sampling 2 or 3)
    int32_t sh_any;         // some instance uses the Shakhov model (the heat-flux kernel runs)
    int32_t all_box;        // every cell is an axis-aligned box and interior neighbours share whole
                            // faces: tracking needs no cell type, and the box of the cell across a
                            // face is this one's with the bounds along the face's axis moved
    int32_t recon_any, recon_all;  // some / every instance reconstructs to second order
    int32_t any_diffuse;           // the mesh has a diffuse wall (the wall kernel runs)
    int32_t count_ch;              // runs of 64 particles per wave of the bucket count (4 or 8)
    const InstP *ip;        // [n_inst]
    InstS *is;              // [n_inst]
    const int32_t *cinst;   // [nc] instance of each cell (n_inst > 1 only)
    long long cap;
    // state
    double *W;              // [5][nc]
    double *P;              // [5][nc] raw particle sums (W^p = P / Omega)
    int32_t *nleft;         // [nc]
    // per-step scratch
    double *tau;            // [nc]
    double *ec;             // [nc] exp(-dt/tau)
    double *rhoh;           // [nc] max(rho - rho^p, 0)
    double *Phi;            // [5][nf]
    double *Wh;             // [5][nc] hydro state (rho^h / rho) W (second order)
    double *gW, *gH;        // [15][nc] limited gradients dW_k/dx_d at [3k+d][nc] (second order)
    double *qh;             // [3][nc] heat flux of the gas (Shakhov model)
    double *S;              // [5][nc] particle sums at the start of the step
    long long *nsam;        // [nc]
    long long *samoff;      // [nc+1]
    long long *scan64;      // scan partials
    long long *ninj;        // [nff] particles entering through each far-field face
    long long *injoff;      // [nff+1]
    int32_t *off;           // [2nc+1]
    int32_t *scan32;        // scan partials
    unsigned long long *spart; // [2][64] crossings and wall hits, spread over 64 slots
    unsigned long long *cnt64; // [2nc] per bucket: stayers << 32 | movers (or collided)
    int32_t *rank;          // [cap + kWallSlack] slot of a mover / collided particle inside its
                            // bucket; during transport, the wall queue (kWallSeg segments)
    unsigned int *wallq;    // [kWallSeg] particles queued in each wall-queue segment
    int32_t *segoff[2];     // [nc+1] each: survivor segments per cell in pa[0] / pa[1]
    int32_t *key;           // [cap]
    int32_t *perm;          // [cap]
    int32_t *big;           // [nc] cells with more than 64 new particles (listed by k_sample)
    Particles pa[2];
    Scalars *sc;
    // time averaging: steps n > avg_from are averaged (avg_from < 0: off)
    long long avg_from;
    double *avgA;           // [5][nc] sum of dt^n W^n over the averaged steps
    double *avgpart;        // [n_inst * kAvgBlocks][2] partial sums of the change and the magnitude
};

}  // namespace ugkwp
