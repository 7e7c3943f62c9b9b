// Internal declarations shared by the libmpm translation units (device + host).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "mpm.h"

namespace mpm {

// ---------------------------------------------------------------- launch shape
constexpr int kThreads = 256;            // 4 wave64 per block
constexpr int kWaves = kThreads / 64;
constexpr int kAlign = 1024;             // unknown counts are padded to this
constexpr long long kLead = 1024;        // zero elements before the first unknown
constexpr int kMaxM = MPM_MAX_RESTART;   // longest restart
constexpr int kMaxSys = 64;              // (problem, species) systems per context
constexpr int kPartRows = 2 * (kMaxM + 1) + 4;   // partial-sum rows per block slot
// warm-start scales on the device: the 5 S + 1 network input channel scales from
// index 0, the S output scales from kScaleOut (room for the largest S)
constexpr int kScaleOut = 5 * MPM_MAX_SPECIES + 1;
constexpr int kScaleCount = kScaleOut + MPM_MAX_SPECIES;
// channels of the warm-start network input: c^n, k, D, s (S each), the mask, and the
// Jacobi-scaled residual of c^n (S)
__host__ __device__ constexpr int ws_channels(int S) { return 5 * S + 1; }
// channels of the static part of that input kept per problem: k, D, s, mask
__host__ __device__ constexpr int ws_static_channels(int S) { return 3 * S + 1; }

// ---------------------------------------------------------------- device views
// Per-problem data, addressed with the problem-local unknown index
// loc = species * Npad + l, where l is the compact index of a domain voxel
// (C order over the box).  Entries with l >= N are zero padding; l == N is the
// "no neighbour" target, always zero.
struct ProbDev {
    const int* vox;        // [Npad] lattice linear index of voxel l (-1 for padding)
    const int4* nbr;       // [Npad] local index of the -y, +y, -z, +z neighbour (N if none)
    const double* d64;     // [S*Npad] A_PP
    const double* q64;     // [S*Npad] dt s + Dirichlet terms (b = c^n + q)
    const double* a64;     // [3][S*Npad] A_PQ toward +x, +y, +z (0 if no coupling)
    const double* sc64;    // [S*Npad] diag(A)^(-1/2) (0 on padding)
    const float* c32;      // [3][S*Npad] scaled S A S couplings toward +x, +y, +z, FP32
    const double* c64;     // [3][S*Npad] the same in FP64
    long long off;         // global index of (species 0, l = 0)
    long long nvox;        // lattice voxel count (species stride of lattice fields)
    int N;                 // domain voxels in the box
    int Npad;              // padded length per species (multiple of kAlign, >= N + 1)
    // geometry for the warm start: lattice (nx, ny), box origin and the box grid the
    // network runs on (box sizes rounded up to multiples of 8)
    int nx, ny;
    int lo[3];
    int gd[3];
    const float* wsout;    // network output on the grid [G][S] (or null)
    uint16_t* wsin;        // network input on the grid [G][5 S + 1], BF16 (or null)
};

// One block of work: a contiguous range of one system's unknowns (global indices),
// with what its kernels need to know about the system up front, so that a block
// reaches its data in one dependent load.
struct Block {
    int sys;     // system id = problem * S + species, -1 for an idle block
    int start;   // global unknown index, multiple of kAlign (relative to kLead)
    int end;
    int slot;    // partial-sum slot of this block
    int slot0;   // first partial-sum slot of the system
    int nb;      // blocks (slots) of the system
    int N;       // domain voxels of the problem
    int tot;     // S * Npad: plane stride of the problem's coupling arrays
    long long base;      // global index of l = 0 of this system
    long long locbase;   // problem-local index of l = 0 (species * Npad)
    const int4* nbr;     // the problem's neighbour table
    const void* c;       // the problem's scaled couplings in the Krylov type
    const double* a64;   // the problem's unscaled couplings (+x, +y, +z planes)
    const double* d64;   // A_PP
    const double* sc64;  // diag(A)^(-1/2)
    const double* q64;   // dt s + Dirichlet terms
    const int* vox;      // lattice index of each compact voxel
    int p, s;            // problem and species of the system
    long long nvox;      // lattice voxels of the problem (species stride of the fields)
    long long pad;
};
static_assert(sizeof(Block) == 128, "block record size");

// Per-system Krylov state.  Within one launch every block reads it and only the
// system's first block writes it, at entries no block of that launch reads.  The
// status fields come first: the host copies only that head of each record
// (kSysHead bytes) between cycles.
struct SysK {
    int active;        // kIdle, kRunning (in a cycle) or kPending (a new cycle starts at step 0)
    int converged;     // true residual met the tolerance this step
    int need_update;   // a cycle finished and x must be corrected
    int mcount;        // basis vectors used by the finished cycle
    int iters, cycles, refinements, breakdown;
    int ws_used, fallback, nblocks, slot0;
    double rel_init, rel_final, rel_warm, kappa_s;
    double h1[kMaxM + 2];    // first Gram-Schmidt coefficients v_k . w
    double h2[kMaxM + 2];    // reorthogonalisation coefficients
    double vs[kMaxM + 2];    // v_k = vs[k] * V_k
    double gt[kMaxM + 2];    // right-hand side entry j before rotation j (read by step j)
    double gf[kMaxM + 2];    // entry j after rotation j (written by step j)
    double cs[kMaxM + 2];    // Givens cosines
    double sn[kMaxM + 2];    // Givens sines
    double y[kMaxM + 2];     // update coefficients of the stored vectors
    double R[(kMaxM + 1) * (kMaxM + 1)];   // column j at R[j * (kMaxM + 1) + i]
    double Hraw[(kMaxM + 1) * (kMaxM + 1)];   // unrotated Hessenberg (delayed Gram-Schmidt)
    double hc[2][kMaxM + 2]; // first-pass coefficients of the column being built (by step parity)
    double bnorm, rnorm, srnorm, eta;
    unsigned long long dmin_bits, dmax_bits;   // extremes of A_PP (positive doubles)
};
constexpr size_t kSysHead = offsetof(SysK, h1);

// Values of SysK::active.  A system whose cycle ended and that needs another one is
// pending until the first kernel of the next cycle (Arnoldi step 0) takes it up, so
// that kernels of later steps launched in the same stretch of work skip it.
constexpr int kIdle = 0, kRunning = 1, kPending = 2;

struct Params {          // per-step scalars read by the kernels
    double tol;
    double inner_rtol;   // floor of the per-cycle reduction (FP32 inner solve)
    int restart;
    int S;
    int first;           // residual kernel: 1 on the first evaluation of a step
    int pad;
};

// Kernel argument bundle of the Krylov kernels.
template <typename T>
struct KArgs {
    const Block* blocks;
    const ProbDev* probs;
    SysK* sk;
    double* part;          // [kPartRows][nslots]
    const Params* prm;
    T* V;                  // basis, vector k at V + k * ldv
    T* W;                  // work vector
    double* x;             // FP64 iterate
    double* b;             // FP64 right-hand side
    double* const* fields; // [P] lattice fields (device pointers)
    SysK* hsk;             // host-visible mirror of the status heads (pinned host memory)
    double* pcur;          // where the gather also writes c^n for the next extrapolation (or null)
    const double* pold;    // c^{n-1} on the global unknowns (extrapolated starts)
    long long ldv;
    int nslots;
    int S;
    int nsys;              // systems of the context (<= 64)
    int pad;
};

// ---------------------------------------------------------------- host helpers
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define MPM_HIP(call)                                          \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return ::mpm::hip_fail(_e, #call); \
    } while (0)

}  // namespace mpm
