// Declarations shared by the C ABI (api.cpp) and the device code (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "coeffs.h"
#include "nflbm.h"

namespace nflbm {

enum StoreKind { kStoreF64 = 0, kStoreF32 = 1, kStoreF16S = 2 };

// Scale applied to binary16 moving populations so that typical magnitudes
// (1e-5 .. 1e-1) stay in the normal range; a power of two, so scaling is exact.
constexpr float kHalfScale = 4096.0f;
// FP16S node records (moment form): binary16 numbers holding the value times
// a power of two, mu~ times kRecMuScale (|mu~| stays below 32: the factored
// flux potential does not depend on the tensions' size, and its Laplacian
// part is bounded by 3 D), (v, -3/2 v.v), (fB, F) and the f moments times
// kRecVelScale (|v| < 0.3 and |P| < 4; a body force of 1e-7 stays normal).
constexpr float kRecMuScale = 2048.0f;
constexpr float kRecVelScale = 16384.0f;

// Per-simulation constants read by every kernel, in the compute precision T.
// Components are in internal order: the evolved ones first (user order kept),
// the implicit one last.
template <class T>
struct DevParams {
  T beta[kMaxComp][kMaxComp];
  T kappa[kMaxComp][kMaxComp];
  T psi[kMaxComp][kMaxComp][kMaxComp];
  T xt[kMaxComp][kMaxComp][kMaxComp];
  T zt[kMaxComp][kMaxComp][kMaxComp];
  T omega_p[kMaxComp];    // 1/tau_i
  T omega_m[kMaxComp];    // TRT odd rate (== omega_p for BGK)
  T inv_tau_g[kMaxComp];
  T m;                    // mobility parameter of g^eq
  T k34D;                 // 3D/4
  T k12D;                 // 12/D
  T omega_stab;           // Omega of xi
  T fb[3];                // body force
  int uidx[kMaxComp];     // user index of internal component i
};

// Tables of the concentration-dependent mobility variant (Appendix C), in
// internal component order and the compute precision T.  The literal flux
// potentials mu_j + phi_j + xi_j need the Lambda and Theta coefficients
// themselves, which the factored tables of DevParams fold away.
template <class T>
struct MobParams {
  T lam[kMaxComp][kMaxComp][kMaxComp][kMaxComp];    // Lambda_{j;klm}: [j][k][l][m], any order of k,l,m
  T theta[kMaxComp][kMaxComp][kMaxComp][kMaxComp];  // Theta_{kl;j;m}: [k][l][j][m], either order of k,l
  T pre[kMaxComp];                                  // (1 - 1/(2 tau_g,i)) m*
};

// Open faces (velocity and concentration Dirichlet, Sec. III C), faces 0..5 =
// x-, x+, y-, y+, z-, z+; internal component order; compute precision T.
template <class T>
struct FaceBC {
  int open;                         // bit f: face f is open (else a wall)
  T fcorr[6][19];                   // 2 w_k (e_k . v_b) / c_s^2, population entering along e_k
  T gsum[6][kMaxComp][19];          // g^eq_k + g^eq_kbar of (C_b, v_b), evolved components
  T cb[6][kMaxComp];                // C_b of every component (stencil value beyond the face)
  T eb[6];                          // E_B(C_b)
};

enum StepFlags {
  kFlagNeedG = 1,         // some tau_g != 1: the update reads g
  kFlagPotential = 2,     // potential-form surface tension
  kFlagOmega = 4,         // Omega != 0
  kFlagMoments = 8,       // moment form of g (tau_g = 1): C, mu~, v, -3/2 v.v per node
  kFlagNoHydro = 16,      // diffusive-only: f not evolved, v = 0
  kFlagCheckNaN = 32,     // this step: the update raises *nanflag at a non-finite node
  kFlagFRecord = 64,      // record form of f (omega+ = omega- = 1): (fB, F) per node
  kFlagFLocal = 128       // moment form, first step after set_fields: the incoming
                          // populations are the initial ones (record form of f: a
                          // node's f is the local equilibrium (A0, v0) of its own
                          // record; g entering across an open face is 0)
};

// What a launch of the update does: a time step, the FP64 node fields of
// the current state (read-back), or their per-workgroup diagnostic sums.
enum UpdateMode { kModeStep = 0, kModeFields = 1, kModeReduce = 2 };

// Device code sees the pointers in the argument structs as pointers to global
// memory, so that it emits global (not flat) accesses and scalar loads for
// uniform reads also where a StepArgs was itself read from memory (batches);
// the host sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define NFLBM_GLOBAL __attribute__((address_space(1)))
#else
#define NFLBM_GLOBAL
#endif

// Population arrays hold post-collision values (pull streaming):
//   f [k-1][node], gk [k-1][node][i], g0 [node][i], conc [node][i], eb [node],
// with the direction strides fstride and gstride below.
// Per-node byte offsets are 32-bit: n times the widest per-node record
// (NE values, the moment form's 4, the mobility variant's N) must stay below 2^32.
struct StepArgs {
  const NFLBM_GLOBAL void* f_src;     // moving hydrodynamic populations
  NFLBM_GLOBAL void* f_dst;
  const NFLBM_GLOBAL void* g0_src;    // rest populations of evolved components
  NFLBM_GLOBAL void* g0_dst;
  const NFLBM_GLOBAL void* gk_src;    // moving populations of evolved components
  NFLBM_GLOBAL void* gk_dst;
  NFLBM_GLOBAL void* conc;            // reconstructed C (compute precision)
  // moment form: the node records of the previous step (C the collision
  // used, mu~ [node][i], and (v, -3/2 v.v) [node][4]); the populations are unused
  const NFLBM_GLOBAL void* cprev;
  NFLBM_GLOBAL void* mu;
  NFLBM_GLOBAL void* vel;
  NFLBM_GLOBAL void* eb;              // E_B per node (compute precision)
  // record form of f: frec [node][4] = (fB, F) of the last collision, with
  // fB = 3 P - 3/2 v.F (after set_fields: (3 P0 - 3/2 v0.v0, v0)),
  // and fmom [node][4] = (sum_k f_k, sum_k e_k f_k) of the streamed f,
  // written by the reconstruction for the update
  NFLBM_GLOBAL void* frec;
  NFLBM_GLOBAL void* fmom;
  NFLBM_GLOBAL double* fields;        // fields-mode output [2N+7][n]
  const NFLBM_GLOBAL void* params;    // DevParams<T>
  // Solid geometry (null without): per node, bit k (1 <= k < Q) set when the
  // population arriving along e_k would come from a solid node or from
  // beyond a wall face, bit 0 set at solid nodes themselves.
  const NFLBM_GLOBAL uint32_t* bb;
  const NFLBM_GLOBAL void* faces;     // FaceBC<T> when some face is open, else null
  // Convective outflow face (-1 none): post-streaming populations of its
  // boundary plane, f [k-1][p] and g [i][k][p] (all k), and the ghost values
  // beyond it, C [i][p] and E_B [NE][p], compute precision, p the in-plane index
  int out_face;
  NFLBM_GLOBAL void* out_f;
  NFLBM_GLOBAL void* out_g;
  NFLBM_GLOBAL void* out_ghost;
  // NaN check (steps with kFlagCheckNaN): set to 1 where a node's C, mu~,
  // v or P is not finite; cleared by the host
  NFLBM_GLOBAL int* nanflag;
  // reduce mode: partial diagnostic records [workgroup][3N + 9], internal
  // component order, and the internal index of the component of v_cm
  NFLBM_GLOBAL double* diag_partial;
  int diag_vcm;
  long long n;
  // distance in elements between the direction arrays of f (f [k-1][node]
  // starts at (k-1) fstride) and of the moving g populations (gk [k-1]
  // starts at (k-1) gstride): an odd multiple of 256 bytes, never a power
  // of two, so that the direction streams fall on different memory channels
  long long fstride, gstride;
  int nx, ny, nz;
  int wall_x, wall_y, wall_z;
  int tx_log2;                        // tile width TX = 1 << tx_log2, TY = 256 / TX
  int zchunk;                         // planes per workgroup (D3Q19)
  int tiles_x, tiles_y, chunks_z;
  // tile column of launch column c (c < tiles_x): tile_x0 + c * tile_xstep,
  // so that one launch can cover a subset of the lattice's tile columns
  int tile_x0, tile_xstep;
  int flags;
};

struct InitArgs {
  void* f; void* g0; void* gk;        // post-collision arrays of the target set
  const double* C;                    // [N][n] user order
  const double* v;                    // [3][n] or null
  const double* P;                    // [n] or null
  const void* params;
  long long n;
  StepArgs sa;                        // lattice size and walls
};

// One step of a batch of simulations that share lattice, N and storage
// precision.  args[m] are the step arguments of member m for this step's
// parity and params[m] its coefficient tables (a DevParams<T> array, T the
// compute precision); a work entry (m, b) is tile b of member m.  The reconstruction's
// tiles are those of one z plane (tiles_x tiles_y nz per member), the update's
// those of its z runs (tiles_x tiles_y chunks_z), all with tile width
// 1 << tx_log2.
struct BatchLaunch {
  const StepArgs* args;               // device [count]
  const void* params;                 // device DevParams<T>[count]
  const int2* work_conc;              // device [blocks_conc] (population form)
  const int2* work_update;            // device [blocks_update]
  int blocks_conc, blocks_update;
  int tx_log2;
  int walls;                          // some member has a wall
  int moments;                        // members use the moment form; the
                                      // reconstruction then runs over the
                                      // update's tiles
  int frecord;                        // members keep f as node records
  int phase;                          // 0 both kernels, 1 the reconstruction
                                      // only, 2 the update only
};

// Arguments of the two kernels of the concentration-dependent mobility
// variant: sa supplies the lattice, walls, the reconstructed C, the new
// population set (gk_dst, g0_dst) and the DevParams; phi is scratch
// [node][N] in the compute precision.
struct MobArgs {
  StepArgs sa;
  const void* mob;                    // MobParams<T>
  void* phi;
};

// The convective outflow's per-step work (after the update, on the new
// state): U from the plane inside the face (partial sums, then U = max(mean,
// 0) in u[0]), then the convected boundary plane and ghosts.  start: capture
// the boundary plane and ghosts of the initial state instead.  A workgroup
// takes kOutNodes plane nodes, its kOutThreads threads splitting each node's
// directions: a plane has few nodes, and the gathers across the face need
// the parallelism.
constexpr int kOutNodes = 64;
constexpr int kOutThreads = 512;
struct OutflowArgs {
  StepArgs sa;
  double* partial;                    // [blocks]
  double* u;                          // [1]
  double fluid;                       // fluid nodes of plane N-1 (U is their mean)
  int blocks;
  int start;                          // 0 convect, 1 capture plane N, 2 refresh plane N's C/E_B/f moments
};

// Launchers: lat 0 = D2Q9, 1 = D3Q19; nc = N; store = StoreKind.
hipError_t launch_conc(int lat, int nc, int store, const StepArgs& a, hipStream_t s);
hipError_t launch_update(int lat, int nc, int store, const StepArgs& a, bool fields, hipStream_t s);
hipError_t launch_init(int lat, int nc, int store, const InitArgs& a, hipStream_t s);
hipError_t launch_batch_step(int lat, int nc, int store, const BatchLaunch& b, hipStream_t s);
hipError_t launch_expand(int lat, int nc, int store, const StepArgs& a, hipStream_t s);
size_t conc_m_lds_bytes(int lat, int nc, int store, int tx_log2, bool frecord);
// Record form of f: the post-collision f of every node written out in the
// population layout (f [k-1][node], direction stride a.fstride, compute
// precision) for read-back; after set_fields (kFlagFLocal) the initial
// equilibria are placed where the first gather pulls them from.
hipError_t launch_expand_f(int lat, int store, const StepArgs& a, void* out, hipStream_t s);
// Diagnostics of the current state without a field buffer: the update in
// reduce mode writes partial records for at most max_blocks workgroups to
// a.diag_partial (returned in *blocks), then one workgroup sums them in a
// fixed order into out [3N + 9] (internal component order).
hipError_t launch_diag(int lat, int nc, int store, const StepArgs& a, int max_blocks, double* out, int* blocks,
                       hipStream_t s);
hipError_t launch_reduce_final(const double* partial, double* out, int N, int blocks, hipStream_t s);
// Domain size (Eq. L): lambda = H(C - 1/2) over [N][n], and partial sums
// [N][blocks][2] of |X|^2 and |k| |X|^2 over an R2C spectrum [N][nc].
hipError_t launch_lambda(const double* C, double* lam, long long total, hipStream_t s);
hipError_t launch_spectrum(const void* X, int N, int nx, int ny, int nz, long long nc, int blocks,
                           double* partial, hipStream_t s);
__host__ __device__ int reduce_record_len(int N);

// Elements between consecutive direction arrays holding `count` elements of
// `esize` bytes each: the bytes rounded up to 256 and then to an odd
// multiple of 256.  With a power-of-two stride (256^3 lattices) the
// direction streams of a node map to the same memory channels; measured at
// 256^3 the update's traffic mix ran 7% faster with the odd stride.
inline size_t direction_stride(size_t count, size_t esize) {
  size_t b = (count * esize + 255) / 256 * 256;
  if ((b / 256) % 2 == 0) b += 256;
  return b / esize;
}

// The diagnostics' reduction grid is capped at this many workgroups, so its
// partial records take at most kDiagMaxBlocks * (3 kMaxComp + 9) doubles.
constexpr int kDiagMaxBlocks = 2048;
// Diagnostics of the current state of s (reconstruction, the update in
// reduce mode, the fixed-order sum) with the partial records at partial
// (max_blocks records) and the summed record at result, both device memory
// the caller provides; fills *out and synchronises.  Allocates nothing.
int diag_run(nflbm_sim* s, int vcm_component, double* partial, int max_blocks, double* result, nflbm_diag* out);
// The device s was created on, and the error path of the C ABI.
int sim_device(const nflbm_sim* s);
int sim_fail(nflbm_sim* s, int code, const char* msg);
size_t update_lds_bytes(int lat, int nc, int store, int tx_log2);
// Concentration-dependent mobility: the literal flux potentials of every node
// (after the reconstruction), and the source term added to the update's
// post-collision populations (after the update).
// Per-node pull masks of StepArgs::bb from a byte mask solid[n] (1 = solid)
// and the wall faces of a.
hipError_t launch_build_bb(int lat, const unsigned char* solid, uint32_t* bb, const StepArgs& a,
                           hipStream_t s);
hipError_t launch_outflow(int lat, int nc, int store, const OutflowArgs& o, hipStream_t s);
hipError_t launch_mob_potentials(int lat, int nc, int store, const MobArgs& a, hipStream_t s);
hipError_t launch_mob_source(int lat, int nc, int store, const MobArgs& a, hipStream_t s);

}  // namespace nflbm
