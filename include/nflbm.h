/*
 * nflbm — per-time-step update of the N-component free-energy lattice
 * Boltzmann method with reduction consistency and global momentum
 * conservation (Rennick, Zhang, Bingert, Krause, Kusumaatmaja,
 * arXiv 2605.22214), on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Every function returns an int
 * status (NFLBM_OK = 0, negative on error) unless stated otherwise; none
 * aborts or exits.  After an error, nflbm_last_error(sim) (or
 * nflbm_last_error(NULL) for errors before a simulation exists) returns a
 * message.  All host arrays passed in are copied during the call; the
 * caller keeps ownership.  Device state is owned by the library.
 *
 * Field layout on the host is C order [component][z][y][x] (x fastest),
 * FP64 whatever the storage precision.  Node index = x + nx (y + ny z).
 */
#ifndef NFLBM_H
#define NFLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NFLBM_MAX_COMP 8
#define NFLBM_ABI_VERSION 11

/* Velocity sets.  D2Q9 as printed in Sec. III; D3Q19 the textbook set
 * (rest 1/3, faces 1/18, edges 1/36) the paper refers to for 3-D. */
enum { NFLBM_D2Q9 = 0, NFLBM_D3Q19 = 1 };

/* Storage precision of the populations.
 *   FP64   populations and arithmetic in double.
 *   FP32   populations and arithmetic in float.
 *   FP16S  moving populations (f_k, g_{i,k}, k >= 1) stored as binary16
 *          scaled by 2^12, rest populations g_{i,0} as float; arithmetic in
 *          float.  The rest population of each component absorbs the
 *          rounding of the moving ones, so node mass is kept to float
 *          rounding.
 * Global reductions (mass, momentum) are always accumulated in double. */
enum { NFLBM_FP64 = 0, NFLBM_FP32 = 1, NFLBM_FP16S = 2 };

enum {
  NFLBM_OK = 0,
  NFLBM_EINVAL = -1,    /* bad argument or configuration                    */
  NFLBM_ESINGULAR = -2, /* a coefficient system (alpha, Lambda, Theta) is singular */
  NFLBM_EUNSTABLE = -3, /* mobility above the linear stability bound        */
  NFLBM_ENOMEM = -4,    /* device or host allocation failed                 */
  NFLBM_EDEVICE = -5,   /* a HIP runtime call failed                        */
  NFLBM_ENUMERIC = -6,  /* a NaN or Inf was found in the state              */
  NFLBM_ENOTSUP = -7    /* combination the library does not support         */
};

/* Readback fields for nflbm_get_field (sizes in doubles, n = nx ny nz):
 *   C      N n   concentrations C_i (zeroth moment of g, Sec. III B)
 *   V      3 n   velocity v (Eq. nmom, rho = 1)
 *   P      n     hydrodynamic pressure (Eq. pres)
 *   F      3 n   total force: surface tension (Eq. Fsnew) + body force
 *   MU     N n   flux potential mu~_i = sum_j alpha_ij (mu_j+phi_j+xi_j) (Eq. MU);
 *                zero for the implicit component
 *   F_RAW  (Q-1) n   populations f_1..f_{Q-1} (f_0 is not stored: no
 *                quantity of the scheme reads it)
 *   G_RAW  N Q n populations g_{i,k}; the implicit component's are zero
 * C, V, P, F and MU are the moments of the current (post-streaming) state,
 * i.e. the values the next collision uses. */
enum {
  NFLBM_FIELD_C = 0,
  NFLBM_FIELD_V = 1,
  NFLBM_FIELD_P = 2,
  NFLBM_FIELD_F = 3,
  NFLBM_FIELD_MU = 4,
  NFLBM_FIELD_F_RAW = 5,
  NFLBM_FIELD_G_RAW = 6
};

/* Option flags. */
enum {
  NFLBM_FLAG_POTENTIAL_FORCE = 1, /* F_s = sum_i mu_i grad C_i (Eq. ststand)
                                     instead of the conservative Eq. Fsnew;
                                     a negative control that drifts          */
  NFLBM_FLAG_ALLOW_UNSTABLE = 2,  /* skip the mobility stability check      */
  NFLBM_FLAG_G_POPULATIONS = 4,   /* keep the populations of g even when every
                                     tau_g = 1 (see "Storage of g" below)      */
  NFLBM_FLAG_NO_HYDRO = 8,        /* diffusive-only (Sec. IV B): the LBE of f is
                                     not evolved, v = 0 and P = 0 everywhere;
                                     only the Cahn-Hilliard LBEs of g step     */
  NFLBM_FLAG_C2C2_MOBILITY = 16,  /* concentration-dependent mobility of
                                     Appendix C, see below                     */
  NFLBM_FLAG_F_POPULATIONS = 32   /* keep the populations of f even when the
                                     record form applies ("Storage of f")      */
};

/* Concentration-dependent mobility (Appendix C, Eqs. mobilconc and
 * glbesource), the comparison variant of Fig. 3(d).  The flux uses the
 * per-node alpha_ij = C_i^2 C_j^2 (i != j), alpha_ii = -sum_{j != i} alpha_ij
 * instead of the constant alpha of Eqs. alpha1/alpha2: g^eq carries no
 * mobility term, and each evolved g gains after its relaxation the source
 * (1 - 1/(2 tau_g,i)) w_k m* e_k.G_i with G_i = sum_j alpha_ij
 * grad(mu_j + phi_j + xi_j) (the same isotropic gradient stencil and wall
 * rule as every other gradient).  Under this flag the config field m is m*
 * (the paper uses 10; M = c_s^2 m* (tau_g - 1/2)), g is kept as populations,
 * the constant-mobility stability check is skipped (alpha is at most 1/16
 * in magnitude per entry here), and the library allocates a scratch array of
 * N values per node in the compute precision for the potentials.  The MU
 * field still reports the constant-alpha flux potential, which this variant
 * does not use.  In a batch such members add their potential and source
 * launches between and after the batch's two kernels, and every member of
 * that batch keeps g as populations. */

/* Storage of g.  With every tau_g = 1 a post-collision population of g is
 * its equilibrium, C_i s_k(v) - w_k m mu~_i (Eqs. glbe, geq), so by default
 * the library keeps per node only the C_i the collision used, mu~_i, v and
 * v.v, and the reconstruction of the next step re-forms the populations from
 * them and takes the rest population directly from Eq. geq: the two forms
 * agree to rounding (the population form writes the rest population as C_i
 * minus its stored moving populations).  Some tau_g != 1, or
 * NFLBM_FLAG_G_POPULATIONS, keeps the 19 (N - 1) populations per node.
 * nflbm_storage_form tells which form a simulation uses. */

/* Storage of f.  When every node relaxes f with omega+ = omega- = 1 (every
 * tau_i = 1 with BGK, or TRT with Lambda^TRT = 1/4) and g is in its moment
 * form, a post-collision population of f is fixed by the node's pressure,
 * velocity and force (Eqs. TRT, FTRT, hydroforce with omega = 1):
 *   f*_k = w_k [3 P + 3 e_k.v + 9/2 (e_k.v)^2 - 3/2 v.v
 *               + 3/2 e_k.F + 9/2 (e_k.v)(e_k.F) - 3/2 v.F],
 * so the library keeps (3 P - 3/2 v.F, F) per node beside the (v, -3/2 v.v)
 * of the moment form of g, instead of the Q - 1 populations;
 * the reconstruction forms the moments sum_k f_k and sum_k e_k f_k of the
 * streamed populations from the neighbours' records (halfway bounce-back at
 * walls and solid nodes) and the update reads those.  This is the same
 * arithmetic as the population form up to rounding; FP64 and FP32 storage
 * only (FP16S keeps its binary16 populations), no open faces or outflow
 * (they need g as populations anyway).  NFLBM_FLAG_F_POPULATIONS keeps the
 * populations; nflbm_f_storage_form tells which form a simulation uses.  The
 * first step after nflbm_set_fields takes each node's f as the equilibrium
 * f^eq(P0, v0) of its own initial record, as the population form stores it. */

/*
 * Problem statement (Sec. II-III).
 *   lattice      NFLBM_D2Q9 (nz must be 1) or NFLBM_D3Q19.
 *   nx, ny, nz   lattice nodes, each >= 1.
 *   wall[a]      0: periodic along axis a (x, y, z); 1: halfway bounce-back
 *                walls half a spacing beyond both faces (Sec. III C).  Stencil
 *                neighbours inside a wall take the centre value.
 *   ncomp        N, 2..NFLBM_MAX_COMP.
 *   implicit_comp  the component not evolved by its own LBE; it follows from
 *                sum_i C_i = 1 (Sec. II, after Eq. CHFlux).  -1 selects the
 *                last component, as in the paper.  An absent component must
 *                not be the implicit one if it is to stay exactly zero.
 *   sigma        N*N row-major pairwise surface tensions: symmetric, zero
 *                diagonal, positive off-diagonal.
 *   width_D      interface width D (the paper uses 4).  beta = 6 sigma/D,
 *                kappa = 3 sigma D/4.
 *   omega_stab   Omega of the stabilising term xi_j (Eq. P); 0 disables.
 *   tau          N hydrodynamic relaxation times, > 1/2; a node takes the
 *                tau of its majority component (Sec. III B), the lowest
 *                index on ties.  omega+ = 1/tau.
 *   trt_magic    Lambda^TRT > 0 selects TRT with omega- from
 *                Lambda = (1/omega+ - 1/2)(1/omega- - 1/2); <= 0 selects BGK.
 *   tau_g        N Cahn-Hilliard relaxation times (> 1/2; the paper uses 1),
 *                or NULL for all 1.
 *   m            mobility parameter of g^eq; M = c_s^2 m (tau_g - 1/2).
 *   body_force   uniform body force density added at every node.
 *   precision    NFLBM_FP64 / NFLBM_FP32 / NFLBM_FP16S.
 *   flags        NFLBM_FLAG_* bits.
 */
typedef struct nflbm_config {
  int lattice;
  int nx, ny, nz;
  int wall[3];
  int ncomp;
  int implicit_comp;
  const double *sigma;
  double width_D;
  double omega_stab;
  const double *tau;
  double trt_magic;
  const double *tau_g;
  double m;
  double body_force[3];
  int precision;
  int flags;
} nflbm_config;

typedef struct nflbm_sim nflbm_sim; /* opaque */

/* Global diagnostics of the current state, FP64 (entries >= N unused):
 *   mass[i]       sum_x C_i
 *   momentum[a]   sum_x (sum_k e_k f_k + F/2)_a
 *   max_abs_c[i]  max_x |C_i|     min_c[i]  min_x C_i
 *   max_sum_dev   max_x |sum_i C_i - 1|
 *   vcm[a]        sum_x C_c v_a / sum_x C_c for c = vcm_component
 *   nan           1 if any population is NaN or Inf */
typedef struct nflbm_diag {
  double mass[NFLBM_MAX_COMP];
  double momentum[3];
  double max_abs_c[NFLBM_MAX_COMP];
  double min_c[NFLBM_MAX_COMP];
  double max_sum_dev;
  double vcm[3];
  int vcm_component;
  int nan;
} nflbm_diag;

/* Validate cfg, compute the coefficient tables (alpha, gamma: Eqs. alpha1,
 * alpha2; Lambda: Eq. ngamma; Theta: the system after Eq. P) on the host in
 * FP64, allocate the device state on the current HIP device and set the
 * state to rest with C_1 = 1.  *out receives the handle.  Per-node arrays
 * are addressed with 32-bit byte offsets: ENOTSUP when the widest of them
 * (N - 1 values a node, 4 for the moment form's velocity record, N for the
 * concentration-dependent mobility's potentials) reaches 2^32 bytes, e.g.
 * above 2^28 nodes for N <= 5 in FP32 with the moment form. */
int nflbm_create(const nflbm_config *cfg, nflbm_sim **out);

/* Release all device and host memory of sim (NULL is ignored). */
void nflbm_destroy(nflbm_sim *sim);

/* Run all subsequent device work of sim on this hipStream_t (NULL = the
 * default stream), e.g. torch.cuda.current_stream().cuda_stream. */
int nflbm_set_stream(nflbm_sim *sim, void *hip_stream);

/* Open face (Sec. III C): turns the wall face `face` (0..5 = x-, x+, y-, y+,
 * z-, z+; its axis must be walled in the configuration; 0..3 in D2Q9) into an
 * inlet / outlet with velocity v_b[3] and concentrations C_b[N] (user order,
 * summing to 1).  A population of f entering across it is the node's own
 * opposite post-collision one plus 2 w_k (e_k . v_b) / c_s^2 (velocity
 * Dirichlet with rho_b = 1, the sign that gives the fluid the face's
 * momentum); one of g is minus its own opposite one plus g^eq_k + g^eq_kbar
 * of (C_b, v_b) (anti-bounce-back with the even part of the equilibrium; the
 * flux potential in it is the bulk one of the uniform state C_b); stencil
 * neighbours beyond the face take C_b and E_B(C_b).  Where a link crosses a
 * wall face and an open face the wall wins, between two open faces the first
 * axis's face.  With solid nodes (nflbm_set_solid), a solid node on the face
 * continues beyond it: a link across the face whose in-face part (the link
 * without its component normal to the face) leads to a solid node is a wall
 * link (bounce-back, centre value), so solid channel walls meet an inlet as
 * wall faces do.  Every storage form of g and f, batch members included; in
 * the moment form the first step after nflbm_set_fields takes g entering
 * across the face as the initial 0.  v_b = C_b = NULL makes the face a wall
 * again.  With an outflow face, a face on another axis must meet the outflow
 * plane only at solid nodes (ENOTSUP otherwise: set the solid nodes first).
 * ENOTSUP with the concentration-dependent mobility.  Call before
 * nflbm_set_fields.  EINVAL for a bad face, an unwalled axis, the outflow
 * face, non-finite values or C_b not summing to 1. */
int nflbm_set_open_face(nflbm_sim *sim, int face, const double *v_b, const double *C_b);

/* Convective outflow (Sec. III C, Eq. convect): turns the wall face `face`
 * (numbered as for nflbm_set_open_face; its axis walled, at least 3 nodes
 * long) into an outlet; -1 removes it.  After streaming, every population q
 * (f and g, every direction) of the boundary plane N becomes
 * (q(N, t) + U q(N-1, t+1)) / (1 + U), q(N, t) the plane's post-streaming
 * values of the previous step and U the mean over plane N-1 of the normal
 * momentum sum_k (e_k . n) f_k after streaming (n the outward normal,
 * without the F/2 term; U = 0 where the mean points inwards).  Stencil
 * neighbours beyond the face take ghost values of C_i and E_B convected the
 * same way, psi(N+1, t+1) = (psi(N+1, t) + U psi(N, t+1)) / (1 + U), from
 * psi(N, 0).  The plane N values, the ghosts and the previous U are state:
 * nflbm_set_fields (and a call here after it) starts them from the current
 * populations, and nflbm_get_state / nflbm_set_state include them (after the
 * populations).  At most one outflow face.  Every storage form of g and f
 * (in the moment form the pulled populations are formed from the node
 * records, as the reconstruction forms them), batch members included.  With
 * solid nodes: they must continue straight through the outflow plane (the
 * same on planes N and N-1; ENOTSUP otherwise), U is the mean over the fluid
 * nodes of plane N-1, and a stencil link across the face whose in-face part
 * leads to a solid node is a wall link.  An open face on another axis must
 * meet the outflow plane only at solid nodes (ENOTSUP otherwise).  ENOTSUP
 * with the concentration-dependent mobility.  Device memory: one plane of
 * (Q-1) + (N-1) Q + N values in the compute precision.  EINVAL for a bad
 * face, an unwalled or too short axis, an open face there, or no fluid node
 * on plane N-1.  Synchronises. */
int nflbm_set_outflow(nflbm_sim *sim, int face);

/* Solid geometry (Sec. III C): solid[n] (node order x fastest, copied; 1 =
 * solid, 0 = fluid) marks nodes of any shape as solid, in addition to the wall
 * faces of the configuration.  Every population a fluid node would pull from
 * a solid node is its own opposite post-collision one instead (halfway
 * bounce-back: the solid surface lies half a link beyond the last fluid
 * node), and every stencil neighbour inside a solid takes the node's own
 * value.  Solid nodes hold no fluid: their concentrations and every field
 * read back as 0, and diagnostics leave them out.  Call before
 * nflbm_set_fields (which fills only the fluid nodes); NULL removes the
 * geometry.  Takes 4 bytes per node of device memory besides the state.
 * Goes with open faces and the outflow face as those describe (ENOTSUP for a
 * mask the outflow face cannot take), and with batch members (the batch
 * picks the change up at its next step).  EINVAL if every node is solid.
 * Synchronises. */
int nflbm_set_solid(nflbm_sim *sim, const unsigned char *solid);

/* Initialise the state from host fields: C (N n, required), v (3 n or NULL
 * for rest), P (n or NULL for 0).  f = f^eq(P, v) for k >= 1; g_{i,0} = C_i,
 * g_{i,k>=1} = 0 for the evolved components.  Reference pressure: with the
 * pressure form of the equilibrium (Eq. feq) a uniform pressure P_ref adds
 * 3 w_k P_ref to every f_k, and no step of the method (streaming, both
 * collisions, bounce-back, open faces, outflow) changes that shift.  The
 * state therefore holds the populations of P - P_ref, P_ref the mean of the
 * given P over the fluid nodes (0 without P), which keeps them small in
 * binary16 storage; nflbm_get_field adds P_ref back to P and to F_RAW.  A
 * checkpoint (nflbm_get_state) holds the shifted populations: restore it
 * into a simulation initialised with the same mean P.  Synchronises. */
int nflbm_set_fields(nflbm_sim *sim, const double *C, const double *v, const double *P);

/* Advance nsteps time steps (Sec. III: collide, stream, boundaries), each one
 * a reconstruction of C and one fused update launch on the sim's stream.
 * Asynchronous: returns after queueing the work, without waiting for it.
 * NaN detection: on every K-th step (nflbm_set_nan_check, default K = 16)
 * the update raises a device flag where a node's C, mu~, v or P is not
 * finite, and nflbm_step queues a copy of that flag to host memory behind
 * its steps.  A call returns ENUMERIC, before queueing anything, once such a
 * copy from an earlier call has arrived with the flag raised, so a NaN is
 * reported by the first nflbm_step after its copy completed; the
 * synchronising calls (nflbm_synchronize, nflbm_step_timed) report it at
 * once.  ENUMERIC stays until nflbm_set_fields or nflbm_set_state replaces
 * the state.  EINVAL for nsteps < 0. */
int nflbm_step(nflbm_sim *sim, long long nsteps);

/* Wait for sim's queued work; ENUMERIC if a checked step has seen a NaN or
 * Inf since the state was last set (see nflbm_step), else OK. */
int nflbm_synchronize(nflbm_sim *sim);

/* Check for non-finite values on every `every`-th step (0 turns the check
 * off; default 16).  The check costs a few operations per node on the
 * steps that take it.  EINVAL for every < 0. */
int nflbm_set_nan_check(nflbm_sim *sim, long long every);

/* Advance nsteps and return, through *ms, the elapsed device time measured
 * with HIP events recorded on the sim's stream around the launches; if
 * ms_update is not NULL also time each update launch separately (events
 * around every update kernel) and return their summed duration.
 * Synchronises; ENUMERIC as nflbm_synchronize. */
int nflbm_step_timed(nflbm_sim *sim, long long nsteps, double *ms, double *ms_update);

/* Advance nsteps and return the summed durations of the reconstruction
 * launches (*ms_conc) and of the update launches (*ms_update), each measured
 * with HIP events recorded on the sim's stream right around the launch.
 * Synchronises; ENUMERIC as nflbm_synchronize. */
int nflbm_step_timed_kernels(nflbm_sim *sim, long long nsteps, double *ms_conc, double *ms_update);

/* Copy one field (NFLBM_FIELD_*) of the current state to host_out (sizes in
 * the field list above).  Synchronises. */
int nflbm_get_field(nflbm_sim *sim, int field, double *host_out);

/* Device memory the state of a simulation with configuration cfg occupies
 * (every array the steps read or write: both f sets, g or the node records,
 * the reconstructed C and E_B), each array rounded up to 256 bytes.  Host-only
 * planning: validates cfg as nflbm_create does (same errors), allocates
 * nothing.  For callers that provide the memory, e.g. a torch tensor. */
int nflbm_device_bytes(const nflbm_config *cfg, size_t *bytes);

/* Move the device state of sim into caller memory: dev_ptr (256-byte
 * aligned) of at least nflbm_device_bytes bytes on sim's device.  The
 * current state is copied over and the library's own arrays are freed; from
 * then on the caller keeps the buffer alive until nflbm_destroy (which does
 * not free it).  Binding again to the same pointer does nothing; binding to
 * another copies the state there.  EINVAL for batch members, a NULL or
 * misaligned pointer, or a short buffer.  Synchronises. */
int nflbm_bind_state(nflbm_sim *sim, void *dev_ptr, size_t bytes);

/* alpha (N*N row-major) and gamma (N) of sim (Eqs. alpha1, alpha2), FP64, in
 * user component order; either pointer may be NULL. */
int nflbm_get_coeffs(const nflbm_sim *sim, double *alpha, double *gamma);

/* Raw state checkpoint: nflbm_state_bytes gives the size, get_state copies
 * the device state (storage precision: f_1..f_{Q-1}, then the populations of
 * g or, in the moment form, the node records C, mu~, (v, -3/2 v.v)) to host_raw,
 * set_state restores it bit for bit.  Synchronise. */
int nflbm_state_bytes(nflbm_sim *sim, size_t *bytes);
int nflbm_get_state(nflbm_sim *sim, void *host_raw);
int nflbm_set_state(nflbm_sim *sim, const void *host_raw);

/* FP64 global diagnostics (see nflbm_diag); vcm_component selects C_c for the
 * centre-of-mass velocity (Sec. V A).  The node fields of the current state
 * (those nflbm_get_field returns) are summed in FP64 where they are formed:
 * each workgroup of the update's reduce mode keeps per-thread sums and
 * reduces them with wavefront shuffles, then one workgroup adds the
 * workgroups' records in a fixed order (results do not depend on timing).
 * A buffer of 2048 (3N + 9) doubles for those records is allocated on the
 * first call and kept.  ENUMERIC (with out filled and out->nan = 1) if a NaN
 * or Inf was found.  Synchronises. */
int nflbm_diagnostics(nflbm_sim *sim, int vcm_component, nflbm_diag *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the diagnostics
 * of nflbm_diagnostics (same kernels, same results) with the reduction's
 * partial records in a fixed device array of the library, (2048 + 1)
 * (3 NFLBM_MAX_COMP + 9) doubles (about 0.5 MiB) that each device holds
 * until the process ends, instead of a buffer allocated on the first call.
 * Calls no hipMalloc or hipFree.  Every call on a device shares that
 * device's array and leaves its records there: calls that overlap on one
 * device (other threads or streams) race.  Every lattice fits, since the
 * reduction grid is capped at 2048 workgroups; a record that did not fit
 * would give ENOTSUP.  EINVAL unless the simulation's device is current;
 * ENUMERIC as nflbm_diagnostics.  Synchronises. */
int nflbm_diagnostics_noalloc(nflbm_sim *sim, int vcm_component, nflbm_diag *out);

/* Characteristic domain size L_i of every component (Eq. L, Sec. IV B) of
 * the current state: lambda_i = H(C_i - 1/2) (taken as C_i > 1/2),
 * S_i(k) = |FFT(lambda_i)|^2 over the lattice's wave vectors k = 2 pi m / n
 * (k = 0 left out), L_i = 2 pi sum S_i / sum |k| S_i, in lattice units.
 * L (N doubles, user order) receives the values; a component with no
 * interface gets 0.  FP64 FFT (hipFFT); buffers and plan are made on the
 * first call and kept.  Synchronises. */
int nflbm_domain_size(nflbm_sim *sim, double *L);

/* Host-only (no device needed): the coefficient tables for N tensions sigma
 * (N*N row-major) and width D.  Any output pointer may be NULL.
 *   alpha  N*N, gamma N                   (Eqs. alpha1, alpha2)
 *   psi    N*N*N  Psi[i][l][m], l < m, l,m != i   (factored bulk + phi)
 *   xtab   N*N*N  X[i][k][l],  k < l, i not in {k,l}  (factored xi)
 *   ztab   N*N*N  Z[i][l][m],  l != i, m not in {i,l} (factored xi)
 * Entries outside the stated index sets are 0. */
int nflbm_coefficients(int N, const double *sigma, double D, double *alpha, double *gamma,
                       double *psi, double *xtab, double *ztab);

/* Launch shape of the update kernel: 256-thread workgroups covering a tile
 * 2^tx_log2 wide (tx_log2 4 or 6: 16 x 16 or 64 x 4 tiles); in D3Q19 each
 * workgroup marches through zchunk planes (1 = a single plane) keeping three
 * planes of concentrations in LDS.  A value <= 0 keeps the current setting.
 * EINVAL if the shape is invalid or its LDS window exceeds the device limit.
 * Results do not depend on the shape.  nflbm_get_launch also reports the
 * device's LDS bytes per workgroup (any output pointer may be NULL).  The
 * default shape (chosen at nflbm_create, and again by nflbm_set_solid until
 * a shape is set here, by nflbm_set_conc_launch or by nflbm_autotune)
 * depends on the lattice, the walls, the solid nodes and the precision.
 * With walls on x alone and no solid nodes, both kernels run the first and
 * last tile columns in their wall variant and the columns between in the
 * periodic one, as two launches. */
int nflbm_set_launch(nflbm_sim *sim, int tx_log2, int zchunk);
int nflbm_get_launch(nflbm_sim *sim, int *tx_log2, int *zchunk, int *lds_limit);
/* The same for the reconstruction kernel (zeroth moment of g, Sec. III B),
 * which has a launch shape of its own: in D3Q19 with g in the moment form it
 * marches along z with one plane of node records in LDS and defaults to
 * z runs that leave about 1024 workgroups, while the update keeps its own.
 * Results do not depend on it. */
int nflbm_set_conc_launch(nflbm_sim *sim, int tx_log2, int zchunk);
int nflbm_get_conc_launch(nflbm_sim *sim, int *tx_log2, int *zchunk);

/* 1 if sim keeps g in the moment form, 0 for populations, negative on error. */
int nflbm_storage_form(const nflbm_sim *sim);
/* Storage form of f (see "Storage of f"): 0 populations, 1 node records;
 * EINVAL for NULL. */
int nflbm_f_storage_form(const nflbm_sim *sim);

/* Bytes moved per lattice-node update by the kernels of one step together,
 * counting every stored population once read and once written plus the
 * reconstructed concentrations (written once, read once); f is left out of a
 * diffusive-only run (it is neither read nor written), and the
 * concentration-dependent mobility adds its potentials (written once, read
 * once), a second read of C and the re-write of the moving populations of g. */
int nflbm_bytes_per_node(nflbm_sim *sim, double *bytes);

/* Launch-shape autotuner: times every shape nflbm_set_launch accepts (tile
 * width 16 or 64; in D3Q19 z runs of 1, 2, 4, ... planes and the whole
 * height) for a few steps each and keeps the one with the fastest update
 * launches, then does the same for the reconstruction's shape
 * (nflbm_set_conc_launch) by the rest of the step.  The halo is one node
 * wide in every shape: the stencils (Eq. gradstencil) reach nearest
 * neighbours only.  The state is copied on the device before the trials and
 * restored afterwards, so results are unchanged.  cache_path (may be NULL)
 * names a text file of earlier choices, one "<key>|<values>" line each, keyed
 * by lattice, N, precision, shape, walls, options and device, with the four
 * values "tx_log2 zchunk conc_tx_log2 conc_zchunk"; a cached choice is
 * applied without timing, a new one is appended.  Synchronises. */
int nflbm_autotune(nflbm_sim *sim, const char *cache_path);

/* ------------------------------------------------------------------------
 * Batches: many independent simulations (each a full problem statement of
 * Secs. II-III with its own size, walls, tensions, relaxation times and
 * mobility) that share lattice, ncomp and precision, advanced together.
 * Every time step of the whole batch is two kernel launches whose workgroups
 * cover the tiles of all members; NFLBM_BATCH_GRAPH replays runs of
 * graph_steps such steps from a captured HIP graph.  Each member is an
 * nflbm_sim owned by the batch: nflbm_batch_member returns it for set_fields,
 * get_field, diagnostics, state I/O, solid nodes, open faces, the outflow
 * face or stepping on its own (never nflbm_destroy it).  A member with an
 * outflow face adds its two outflow launches after each batch step; one with
 * the concentration-dependent mobility its potential launch between the
 * batch's two kernels and its source launch after them.  All members run on
 * the batch's stream.
 * ---------------------------------------------------------------------- */
typedef struct nflbm_batch nflbm_batch; /* opaque */

/* Stepping modes. */
enum {
  NFLBM_BATCH_LAUNCH = 0,  /* two launches per step for the whole batch          */
  NFLBM_BATCH_GRAPH = 1,   /* the same launches replayed from a HIP graph         */
  NFLBM_BATCH_PER_SIM = 2  /* each member's own launch sequence, one after another
                              (the reference point the batch is measured against) */
};

/* Create count members from cfgs[0..count) (copied).  EINVAL if count < 1 or
 * the members differ in lattice, ncomp or precision; any error of
 * nflbm_create, prefixed with the member index.  Members start at rest with
 * C_1 = 1, as from nflbm_create.  *out receives the handle. */
int nflbm_batch_create(const nflbm_config *cfgs, int count, nflbm_batch **out);
/* Release the batch and all its members (NULL is ignored). */
void nflbm_batch_destroy(nflbm_batch *b);
/* Number of members (0 for NULL). */
int nflbm_batch_count(const nflbm_batch *b);
/* Borrowed handle of member idx, or NULL (with an error on b) if out of range. */
nflbm_sim *nflbm_batch_member(nflbm_batch *b, int idx);
/* Run the batch and its members on this hipStream_t; NULL returns to the
 * batch's own stream (the legacy default stream cannot be captured). */
int nflbm_batch_set_stream(nflbm_batch *b, void *hip_stream);
/* nflbm_set_fields / nflbm_get_field of member idx. */
int nflbm_batch_set_fields(nflbm_batch *b, int idx, const double *C, const double *v, const double *P);
int nflbm_batch_get_field(nflbm_batch *b, int idx, int field, double *host_out);
/* Advance every member nsteps time steps in mode NFLBM_BATCH_*.  The result
 * is bit-for-bit that of stepping each member alone.  Asynchronous.  In the
 * launch and graph modes every step checks for non-finite values (a captured
 * graph replays one argument table), with one flag for the whole batch
 * reported as nflbm_step reports its own: ENUMERIC from the first call after
 * the flag's copy arrived raised, until nflbm_batch_set_fields; the per
 * simulation mode uses each member's own check. */
int nflbm_batch_step(nflbm_batch *b, long long nsteps, int mode);
/* As nflbm_batch_step, returning in *ms the device time between HIP events
 * recorded on the batch stream before and after.  Synchronises. */
int nflbm_batch_step_timed(nflbm_batch *b, long long nsteps, int mode, double *ms);
/* Tile width 2^tx_log2 (4 or 6) used for every member in the batch launches,
 * and steps per captured graph (even, >= 2); values <= 0 keep the current
 * setting.  Discards captured graphs when the shape changes.  Synchronises. */
int nflbm_batch_set_launch(nflbm_batch *b, int tx_log2, int graph_steps);
int nflbm_batch_get_launch(nflbm_batch *b, int *tx_log2, int *graph_steps, int *blocks_update);
/* Total lattice nodes over all members. */
int nflbm_batch_nodes(const nflbm_batch *b, long long *nodes);
/* Autotuner of the batch tile width (graph mode), as nflbm_autotune; the cache
 * key adds the member count, node total and a hash of the member shapes. */
int nflbm_batch_autotune(nflbm_batch *b, const char *cache_path);
/* Message of the last error on b (of the calling thread if b is NULL). */
const char *nflbm_batch_last_error(const nflbm_batch *b);

/* Message of the last error on sim (or of the calling thread if sim is NULL).
 * The pointer stays valid until the next call on the same sim / thread. */
const char *nflbm_last_error(const nflbm_sim *sim);

/* NFLBM_ABI_VERSION of the built library. */
int nflbm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NFLBM_H */
