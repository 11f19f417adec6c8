// C ABI of the N-component free-energy LBM library (see include/nflbm.h).
#include "nflbm.h"

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "coeffs.h"
#include "internal.h"

using namespace nflbm;

namespace {

thread_local std::string g_thread_error;

// Velocity sets (the same ordering as the device code: opposite directions
// adjacent, k + 1 for odd k).
constexpr int kD2Q9[19][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                              {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
constexpr int kD3Q19[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
constexpr double kW2[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
constexpr double kW3[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

}  // namespace

struct nflbm_sim {
  // problem
  int lat = 0, N = 0, NE = 0, Q = 0, store = 0, flags = 0;
  int nx = 0, ny = 0, nz = 0, wall[3] = {0, 0, 0};
  int implicit = 0;
  int uidx[kMaxComp] = {};  // internal -> user component
  size_t n = 0;
  Coeffs co;
  // storage sizes (bytes per value), and the elements between direction
  // arrays of f and of the moving g populations (direction_stride)
  size_t fs = 0, g0s = 0, ts = 0;
  size_t rs = 0;   // bytes of a node-record value of the moment form (mu~, v, f records)
  size_t fstride = 0, gstride = 0;
  // device state: two population sets (A/B), reconstructed C, parameters
  void* f[2] = {nullptr, nullptr};
  void* g0[2] = {nullptr, nullptr};
  void* gk[2] = {nullptr, nullptr};
  // reconstructed C: one array (population form), or the two records of the
  // moment form (the collision's C of the current state, and the next C)
  void* conc[2] = {nullptr, nullptr};
  void* mu = nullptr;    // moment form: mu~ [node][i]
  void* vel = nullptr;   // moment form: (v, -3/2 v.v) [node][4]
  int gform = 0;         // 0 populations of g, 1 moment form (tau_g = 1)
  // record form of f (every omega+ = omega- = 1, with the moment form of g):
  // frec (fB, F) [node][4] instead of the f populations, fmom [node][4] the
  // moments of the streamed f; f_local: the next step starts from the
  // equilibria set_fields wrote (each node's own record)
  int fform = 0;
  void* frec = nullptr;
  void* fmom = nullptr;
  bool f_local = false;
  // open faces: FaceBC<T> on the device, and the host's copy of each face
  void* faces = nullptr;
  int open_mask = 0;
  double face_v[6][3] = {};
  double face_c[6][kMaxComp] = {};   // user order
  double m_geq = 0.0, omega = 0.0;
  // Reference pressure: the state holds the populations of P - p_ref (the
  // mean initial P of the fluid nodes); read-back adds it to P and F_RAW
  double p_ref = 0.0;
  // convective outflow face (-1 none): one device block holding the plane
  // buffers f [Q-1][P], g [N-1][Q][P] and the ghosts [N][P] (compute
  // precision), and the per-workgroup momentum sums plus U (FP64)
  int out_face = -1;
  size_t out_plane = 0;
  double out_fluid = 0.0;   // fluid nodes of plane N-1 (U is their mean)
  void* out_buf = nullptr;
  double* out_red = nullptr;
  int out_blocks = 0;
  // solid geometry: per-node pull masks (StepArgs::bb) and the caller's mask
  uint32_t* bb = nullptr;
  std::vector<unsigned char> solid_host;
  // concentration-dependent mobility: MobParams and the potential scratch
  bool c2c2 = false;
  void* mob = nullptr;
  void* phi = nullptr;
  bool borrowed = false; // state arrays live in caller memory (nflbm_bind_state)
  // domain-size diagnostic: batched R2C plan and its buffers (made on first use)
  hipfftHandle fft = 0;
  bool fft_made = false;
  double* lam = nullptr;
  void* spec = nullptr;
  double* spart = nullptr;
  bool in_batch = false;
  // incremented by every change of solid nodes, open faces or the outflow
  // face: a batch rebuilds its step arguments (and drops its graphs) when a
  // member's count differs from the one its tables were built for
  unsigned boundary_version = 0;
  void* eb = nullptr;
  void* params = nullptr;
  double* fields = nullptr;
  double* red = nullptr;
  int cur = 0;
  hipStream_t stream = nullptr;
  // launch shape of the update, and of the reconstruction (its own: the two
  // kernels measured fastest with different tiles)
  int tx_log2 = 6, zchunk = 1, tiles_x = 1, tiles_y = 1, chunks_z = 1;
  int ctx_log2 = 6, czchunk = 1, ctiles_x = 1, ctiles_y = 1, cchunks_z = 1;
  // a shape set by the caller or the autotuner, kept when solid nodes come or go
  bool shape_chosen = false;
  size_t lds_max = 65536;
  int step_flags = 0;
  int device = 0;        // the HIP device current at nflbm_create
  // NaN detection: the update raises *nanflag on the steps it checks (every
  // nan_every-th step, 0 = never); nflbm_step copies the flag to pinned host
  // memory behind the checked steps and reads the copy, once its event has
  // completed, on the next call (no synchronisation on the stepping path)
  int* nanflag = nullptr;
  int* nan_host = nullptr;
  hipEvent_t nan_ev = nullptr;
  bool nan_pending = false;
  int nan_seen = 0;
  long long nan_every = 16;
  long long step_count = 0;
  std::string err;
};

struct nflbm_batch {
  std::vector<nflbm_sim*> members;
  int lat = 0, N = 0, store = 0;
  int walls = 0;
  long long nodes = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  // launch shape shared by all members
  int tx_log2 = 6;
  int graph_steps = 32;
  // device: step arguments for the two parities [2][count], coefficient
  // tables [count], work lists
  StepArgs* args = nullptr;
  void* params = nullptr;
  int2* work_conc = nullptr;
  int2* work_update = nullptr;
  int blocks_conc = 0, blocks_update = 0;
  std::vector<int> key;     // member parities that args[0..count) was built for
  std::vector<unsigned> versions;   // members' boundary_version at that build
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  // NaN flag shared by the members' batch steps, which check every step
  // (a captured graph replays one argument table); host copy as for a sim
  int* nanflag = nullptr;
  int* nan_host = nullptr;
  hipEvent_t nan_ev = nullptr;
  bool nan_pending = false;
  int nan_seen = 0;
  std::string err;
};

namespace {

int fail(nflbm_sim* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  else g_thread_error = msg;
  return code;
}

int hip_fail(nflbm_sim* s, hipError_t e, const char* what) {
  return fail(s, NFLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(sim, call)                              \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(sim, e_, #call); \
  } while (0)

template <class T>
void fill_params(const nflbm_sim& s, const double* tau, const double* tau_g, double trt,
                 double m, double omega, const double* fb, DevParams<T>* p) {
  std::memset(p, 0, sizeof(*p));
  const int N = s.N;
  const Coeffs& c = s.co;
  for (int i = 0; i < N; ++i) {
    const int ui = s.uidx[i];
    p->uidx[i] = ui;
    for (int j = 0; j < N; ++j) {
      const int uj = s.uidx[j];
      p->beta[i][j] = static_cast<T>(c.beta[ui][uj]);
      p->kappa[i][j] = static_cast<T>(c.kappa[ui][uj]);
      for (int k = 0; k < N; ++k) {
        const int uk = s.uidx[k];
        const int lo = uj < uk ? uj : uk, hi = uj < uk ? uk : uj;
        if (j != k && j != i && k != i) {
          p->psi[i][j][k] = static_cast<T>(c.psi[ui][lo][hi]);
          p->xt[i][j][k] = static_cast<T>(c.xt[ui][lo][hi]);
        }
        if (j != i && k != i && k != j) p->zt[i][j][k] = static_cast<T>(c.zt[ui][uj][uk]);
      }
    }
    const double t = tau[ui];
    const double wp = 1.0 / t;
    const double wm = trt > 0.0 ? 1.0 / (0.5 + trt / (t - 0.5)) : wp;
    p->omega_p[i] = static_cast<T>(wp);
    p->omega_m[i] = static_cast<T>(wm);
    p->inv_tau_g[i] = static_cast<T>(1.0 / (tau_g ? tau_g[ui] : 1.0));
  }
  p->m = static_cast<T>(m);
  p->k34D = static_cast<T>(0.75 * c.D);
  p->k12D = static_cast<T>(12.0 / c.D);
  p->omega_stab = static_cast<T>(omega);
  for (int d = 0; d < 3; ++d) p->fb[d] = static_cast<T>(fb[d]);
}

void free_device(nflbm_sim* s) {
  void** arrays[] = {&s->f[0], &s->f[1], &s->g0[0], &s->g0[1], &s->gk[0], &s->gk[1],
                     &s->conc[0], &s->conc[1], &s->mu, &s->vel, &s->eb, &s->frec, &s->fmom};
  for (void** a : arrays) {
    if (*a && !s->borrowed) (void)hipFree(*a);
    *a = nullptr;
  }
  if (s->params) (void)hipFree(s->params);
  if (s->bb) (void)hipFree(s->bb);
  s->bb = nullptr;
  if (s->faces) (void)hipFree(s->faces);
  s->faces = nullptr;
  if (s->out_buf) (void)hipFree(s->out_buf);
  if (s->out_red) (void)hipFree(s->out_red);
  s->out_buf = nullptr;
  s->out_red = nullptr;
  if (s->mob) (void)hipFree(s->mob);
  if (s->phi) (void)hipFree(s->phi);
  s->mob = s->phi = nullptr;
  if (s->fft_made) (void)hipfftDestroy(s->fft);
  s->fft_made = false;
  if (s->lam) (void)hipFree(s->lam);
  if (s->spec) (void)hipFree(s->spec);
  if (s->spart) (void)hipFree(s->spart);
  s->lam = nullptr;
  s->spec = nullptr;
  s->spart = nullptr;
  if (s->fields) (void)hipFree(s->fields);
  if (s->red) (void)hipFree(s->red);
  s->params = s->eb = nullptr;
  s->fields = s->red = nullptr;
  if (s->nanflag) (void)hipFree(s->nanflag);
  if (s->nan_host) (void)hipHostFree(s->nan_host);
  if (s->nan_ev) (void)hipEventDestroy(s->nan_ev);
  s->nanflag = nullptr;
  s->nan_host = nullptr;
  s->nan_ev = nullptr;
}

int next_pow2_log(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

size_t device_lds_max() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
      prop.sharedMemPerBlock > 0)
    return prop.sharedMemPerBlock;
  return 65536;
}

// Apply a launch shape; returns false if it is invalid or its LDS does not fit.
bool apply_launch(nflbm_sim* s, int l, int zc) {
  if (l != 4 && l != 6) return false;
  if (s->lat != NFLBM_D3Q19) zc = 1;
  if (zc < 1) return false;
  if (zc > s->nz) zc = s->nz;
  if (update_lds_bytes(s->lat, s->N, s->store, l) > s->lds_max) return false;
  if (s->gform && conc_m_lds_bytes(s->lat, s->N, s->store, l, s->fform) > s->lds_max) return false;
  const int TX = 1 << l, TY = 256 >> l;
  s->tx_log2 = l;
  s->zchunk = zc;
  s->tiles_x = (s->nx + TX - 1) / TX;
  s->tiles_y = (s->ny + TY - 1) / TY;
  s->chunks_z = s->lat == NFLBM_D3Q19 ? (s->nz + zc - 1) / zc : 1;
  return true;
}

// Launch shape of the reconstruction; false if invalid or its LDS does not fit.
bool apply_conc_launch(nflbm_sim* s, int l, int zc) {
  if (l != 4 && l != 6) return false;
  if (s->lat != NFLBM_D3Q19) zc = 1;
  if (zc < 1) return false;
  if (zc > s->nz) zc = s->nz;
  if (s->gform && conc_m_lds_bytes(s->lat, s->N, s->store, l, s->fform) > s->lds_max) return false;
  const int TX = 1 << l, TY = 256 >> l;
  s->ctx_log2 = l;
  s->czchunk = zc;
  s->ctiles_x = (s->nx + TX - 1) / TX;
  s->ctiles_y = (s->ny + TY - 1) / TY;
  s->cchunks_z = s->lat == NFLBM_D3Q19 ? (s->nz + zc - 1) / zc : 1;
  return true;
}

// z run per workgroup that leaves about `target` workgroups for tile width 1 << l.
int zchunk_for(const nflbm_sim* s, int l, long long target) {
  if (s->lat != NFLBM_D3Q19) return 1;
  const int TX = 1 << l, TY = 256 >> l;
  const long long xy = static_cast<long long>((s->nx + TX - 1) / TX) * ((s->ny + TY - 1) / TY);
  long long chunks = target / (xy > 0 ? xy : 1);
  if (chunks < 1) chunks = 1;
  if (chunks > s->nz) chunks = s->nz;
  int zc = static_cast<int>((s->nz + chunks - 1) / chunks);
  if (zc < 4) {
    // runs shorter than 4 planes re-load more halo planes; they are taken
    // only where 4-plane runs would leave too few workgroups to fill the
    // chip (a 16 x 16 x 192 channel: 48 workgroups of 4 planes, 192 of one)
    const int zc4 = s->nz < 4 ? s->nz : 4;
    if (xy * ((s->nz + zc4 - 1) / zc4) >= 1024) zc = zc4;
  }
  return zc;
}

// Default shapes.  Update: tiles 64 x 4 (16 x 16 when nx <= 16 or when the
// wider LDS window does not fit), in 3-D a z run per workgroup that leaves
// about 8192 workgroups (4096 in the float record form of f, whose update
// prefetches across the run: runs of 16 against 8 planes measured 0.303
// against 0.314 ms at 256^3; 1024 in FP64, where longer runs measured
// faster).
// Reconstruction: the update's tile width; in the moment form's 3-D z march a
// run that leaves about 1024 workgroups (each run re-loads two planes beyond
// its ends, so long runs pay off as long as the CUs stay busy: 0.255 ms at
// 256^3 in FP32 against 0.262 ms for 8192 workgroups); otherwise about 4096
// (1024 in FP64).
// Uses the LDS limit already in s->lds_max.
int default_launch(nflbm_sim* s) {
  auto fits = [&](int t) {
    return update_lds_bytes(s->lat, s->N, s->store, t) <= s->lds_max &&
           (!s->gform || conc_m_lds_bytes(s->lat, s->N, s->store, t, s->fform) <= s->lds_max);
  };
  int l = s->nx <= 16 ? 4 : 6;
  if (l == 6 && !fits(l)) l = 4;
  if (!fits(l)) return -1;
  // Walls on x in D3Q19, in float: the update's z runs leave about 2048
  // workgroups (runs of 8 planes at 256 x 128 x 128, 64-wide tiles: inlet +
  // outflow 0.093 -> 0.087 ms and solid posts 0.116 -> 0.111 ms against the
  // 16 x 16 tiles with runs of 4 taken before the wall variants prefetched).
  // With walls on x alone and no solid nodes, and at least three 64-wide tile
  // columns, both kernels run their edge columns in the wall variant and the
  // columns between in the periodic one (split_x_walls), two launches that
  // each need workgroups of their own: the reconstruction's runs then also
  // leave about 2048 workgroups over the two (0.171 -> 0.125 ms against the
  // runs of 16 that 1024 give).
  const bool xw = s->lat == NFLBM_D3Q19 && s->wall[0];
  const bool split = xw && !s->wall[1] && !s->wall[2] && !s->bb && (s->nx + 63) / 64 >= 3;
  const bool f64 = s->store == NFLBM_FP64;
  const long long tu = f64 ? 1024 : xw ? 2048 : (s->fform ? 4096 : 8192);
  const long long tc = f64 ? 1024 : split ? 2048 : (s->gform ? 1024 : 4096);
  if (!apply_launch(s, l, zchunk_for(s, l, tu))) return -1;
  return apply_conc_launch(s, l, zchunk_for(s, l, tc)) ? 0 : -1;
}

int choose_launch(nflbm_sim* s) {
  s->lds_max = device_lds_max();
  return default_launch(s);
}

// The step arguments with the reconstruction's launch shape.
StepArgs conc_args(const nflbm_sim* s, const StepArgs& a) {
  StepArgs c = a;
  c.tx_log2 = s->ctx_log2;
  c.zchunk = s->czchunk;
  c.tiles_x = s->ctiles_x;
  c.tiles_y = s->ctiles_y;
  c.chunks_z = s->cchunks_z;
  return c;
}

StepArgs make_args(const nflbm_sim* s, int src) {
  StepArgs a{};
  a.f_src = s->f[src];
  a.f_dst = s->f[1 - src];
  if (s->gform) {
    a.cprev = s->conc[src];
    a.conc = s->conc[1 - src];
    a.mu = s->mu;
    a.vel = s->vel;
  } else {
    a.g0_src = s->g0[src];
    a.g0_dst = s->g0[1 - src];
    a.gk_src = s->gk[src];
    a.gk_dst = s->gk[1 - src];
    a.conc = s->conc[0];
  }
  a.eb = s->eb;
  a.frec = s->frec;
  a.fmom = s->fmom;
  a.nanflag = s->nanflag;
  a.fields = s->fields;
  a.params = s->params;
  a.bb = s->bb;
  a.faces = s->faces;
  a.out_face = s->out_face;
  if (s->out_face >= 0) {
    const size_t P = s->out_plane;
    unsigned char* b = static_cast<unsigned char*>(s->out_buf);
    a.out_f = b;
    a.out_g = b + size_t(s->Q - 1) * P * s->ts;
    a.out_ghost = b + (size_t(s->Q - 1) + size_t(s->NE) * s->Q) * P * s->ts;
  }
  a.n = static_cast<long long>(s->n);
  a.fstride = static_cast<long long>(s->fstride);
  a.gstride = static_cast<long long>(s->gstride);
  a.nx = s->nx;
  a.ny = s->ny;
  a.nz = s->nz;
  a.wall_x = s->wall[0];
  a.wall_y = s->wall[1];
  a.wall_z = s->wall[2];
  a.tx_log2 = s->tx_log2;
  a.zchunk = s->zchunk;
  a.tiles_x = s->tiles_x;
  a.tiles_y = s->tiles_y;
  a.chunks_z = s->chunks_z;
  a.tile_xstep = 1;
  a.flags = s->step_flags;
  if (s->gform && s->f_local) a.flags |= kFlagFLocal;
  return a;
}

int ensure_fields(nflbm_sim* s) {
  if (!s->fields) {
    const size_t bytes = size_t(2 * s->N + 7) * s->n * sizeof(double);
    if (hipMalloc(reinterpret_cast<void**>(&s->fields), bytes) != hipSuccess) {
      s->fields = nullptr;
      return fail(s, NFLBM_ENOMEM, "cannot allocate the readback field buffer");
    }
  }
  return NFLBM_OK;
}

// Tables of the concentration-dependent mobility in internal component order:
// Lambda and Theta are symmetric in their index sets, so every ordering of a
// set is filled from the sorted user-index entry.
template <class T>
void fill_mob(const nflbm_sim& s, const double* tau_g, double m_star, MobParams<T>* p) {
  std::memset(p, 0, sizeof(*p));
  const int N = s.N;
  const Coeffs& c = s.co;
  auto srt = [](int* v, int n) {
    for (int x = 0; x < n; ++x)
      for (int y = x + 1; y < n; ++y)
        if (v[y] < v[x]) std::swap(v[x], v[y]);
  };
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < N; ++k)
      for (int l = 0; l < N; ++l)
        for (int m = 0; m < N; ++m) {
          const int uj = s.uidx[j];
          int t[3] = {s.uidx[k], s.uidx[l], s.uidx[m]};
          if (k != l && k != m && l != m && j != k && j != l && j != m) {
            srt(t, 3);
            p->lam[j][k][l][m] = static_cast<T>(c.lam[uj][t[0]][t[1]][t[2]]);
          }
          // theta[k][l][j][m]: pair {k, l}, then j and m outside it
          if (k != l && j != k && j != l && m != k && m != l && m != j) {
            int pr[2] = {s.uidx[k], s.uidx[l]};
            srt(pr, 2);
            p->theta[k][l][j][m] = static_cast<T>(c.theta[pr[0]][pr[1]][uj][s.uidx[m]]);
          }
        }
  for (int i = 0; i < N; ++i) {
    const double tg = tau_g ? tau_g[s.uidx[i]] : 1.0;
    p->pre[i] = static_cast<T>((1.0 - 0.5 / tg) * m_star);
  }
}

// Convective outflow of the state set `cur`.  mode 0 convects after a step,
// 1 captures the boundary plane of the current state, 2 only re-derives plane
// N's C, E_B and f moments from the plane buffers (moment form).
OutflowArgs outflow_args(const nflbm_sim* s, int cur, int mode) {
  OutflowArgs o{};
  o.sa = make_args(s, cur);
  // after a step the plane N-1 populations are the streamed ones (the
  // first-step flag of the moment form describes only the state before it)
  if (mode == 0) o.sa.flags &= ~kFlagFLocal;
  o.partial = s->out_red;
  o.u = s->out_red + s->out_blocks;
  o.fluid = s->out_fluid;
  o.blocks = s->out_blocks;
  o.start = mode;
  return o;
}

int launch_outflow_step(nflbm_sim* s, int mode) {
  HIPCHK(s, launch_outflow(s->lat, s->N, s->store, outflow_args(s, s->cur, mode), s->stream));
  return NFLBM_OK;
}

// In the moment form the reconstruction leaves C, E_B and the f moments of
// the outflow plane to the outflow kernel, which writes them into arrays that
// are not part of the state: after the state is replaced they are re-derived
// from the restored plane buffers.
int refresh_outflow_plane(nflbm_sim* s) {
  if (s->out_face < 0 || !s->gform) return NFLBM_OK;
  return launch_outflow_step(s, 2);
}

size_t out_buf_bytes(const nflbm_sim* s) {
  return (size_t(s->Q - 1) + size_t(s->NE) * s->Q + size_t(s->N)) * s->out_plane * s->ts;
}

MobArgs mob_args(const nflbm_sim* s, const StepArgs& a) {
  MobArgs m{};
  m.sa = a;
  m.mob = s->mob;
  m.phi = s->phi;
  return m;
}

// One time step from state set `cur`; ev (optional) brackets the update.
// Every nan_every-th step the update checks for non-finite values (*checked
// is set when this one did).
int launch_step(nflbm_sim* s, hipEvent_t ev0, hipEvent_t ev1, bool* checked = nullptr, hipEvent_t evc0 = nullptr,
                hipEvent_t evc1 = nullptr) {
  StepArgs a = make_args(s, s->cur);
  ++s->step_count;
  if (s->nan_every > 0 && s->step_count % s->nan_every == 0) {
    a.flags |= kFlagCheckNaN;
    if (checked) *checked = true;
  }
  if (evc0) HIPCHK(s, hipEventRecord(evc0, s->stream));
  HIPCHK(s, launch_conc(s->lat, s->N, s->store, conc_args(s, a), s->stream));
  if (evc1) HIPCHK(s, hipEventRecord(evc1, s->stream));
  if (s->c2c2) HIPCHK(s, launch_mob_potentials(s->lat, s->N, s->store, mob_args(s, a), s->stream));
  if (ev0) HIPCHK(s, hipEventRecord(ev0, s->stream));
  HIPCHK(s, launch_update(s->lat, s->N, s->store, a, false, s->stream));
  if (ev1) HIPCHK(s, hipEventRecord(ev1, s->stream));
  if (s->c2c2) HIPCHK(s, launch_mob_source(s->lat, s->N, s->store, mob_args(s, a), s->stream));
  s->cur ^= 1;
  s->f_local = false;   // from now on every f streams in from its neighbour
  if (s->out_face >= 0) return launch_outflow_step(s, 0);
  return NFLBM_OK;
}

// Host copy of a NaN flag behind the work queued so far on stream.
hipError_t nan_enqueue(int* dev, int* host, hipEvent_t ev, hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(host, dev, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipEventRecord(ev, stream);
  return e;
}

// Read the host copy of a NaN flag if its copy has completed (wait: block
// until it has); *seen becomes 1, and stays so, once a NaN was reported.
hipError_t nan_poll(bool* pending, int* seen, const int* host, hipEvent_t ev, bool wait) {
  if (!*pending) return hipSuccess;
  hipError_t e = wait ? hipEventSynchronize(ev) : hipEventQuery(ev);
  if (e == hipErrorNotReady) return hipSuccess;
  if (e != hipSuccess) return e;
  *pending = false;
  if (*host) *seen = 1;
  return hipSuccess;
}

int sim_nan_status(nflbm_sim* s, bool wait) {
  HIPCHK(s, nan_poll(&s->nan_pending, &s->nan_seen, s->nan_host, s->nan_ev, wait));
  if (s->nan_seen) return fail(s, NFLBM_ENUMERIC, "a NaN or Inf appeared in the state (checked steps)");
  return NFLBM_OK;
}

// Clear the NaN flag of s (with the state it refers to).
int sim_nan_reset(nflbm_sim* s) {
  HIPCHK(s, hipStreamSynchronize(s->stream));
  HIPCHK(s, hipMemset(s->nanflag, 0, sizeof(int)));
  *s->nan_host = 0;
  s->nan_pending = false;
  s->nan_seen = 0;
  return NFLBM_OK;
}

// Bulk flux potential mu~_i of a uniform state C (user order, Laplacian 0):
// the factored form of Eq. MU with the tables of coeffs.cpp.
double mu_bulk(const Coeffs& c, const double* C, double omega, int i) {
  const int N = c.N;
  double br = -(1.0 - 3.0 * C[i] + 2.0 * C[i] * C[i]);
  for (int l = 0; l < N; ++l)
    for (int m = l + 1; m < N; ++m)
      if (l != i && m != i) br += c.psi[i][l][m] * C[l] * C[m];
  double val = (12.0 / c.D) * C[i] * br;
  if (omega != 0.0) {
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < N; ++k)
      for (int l = k + 1; l < N; ++l)
        if (k != i && l != i) sx += c.xt[i][k][l] * C[k] * C[k] * C[l] * C[l];
    for (int l = 0; l < N; ++l) {
      if (l == i) continue;
      double inner = 0.0;
      for (int m = 0; m < N; ++m)
        if (m != i && m != l) inner += c.zt[i][l][m] * C[m];
      sy += C[l] * C[l] * inner;
    }
    val += (12.0 / c.D) * omega * C[i] * (sx + C[i] * sy);
  }
  return val;
}

double bulk_energy_host(const Coeffs& c, const double* C) {
  auto fp = [](double x) { return x * x * (1.0 - x) * (1.0 - x); };
  double e = 0.0;
  for (int i = 0; i < c.N; ++i)
    for (int j = i + 1; j < c.N; ++j) e += c.beta[i][j] * (fp(C[i]) + fp(C[j]) - fp(C[i] + C[j]));
  return e;
}

// Open-face terms of fill_faces in FP64, for the host's read-back of the
// post-streaming populations: f correction and g^eq_k + g^eq_kbar of
// component u (user index) for the population entering along e_k.
double face_fcorr(const nflbm_sim& s, int f, int k) {
  const int (*E)[3] = s.lat == NFLBM_D2Q9 ? kD2Q9 : kD3Q19;
  const double* W = s.lat == NFLBM_D2Q9 ? kW2 : kW3;
  const double* v = s.face_v[f];
  return 6.0 * W[k] * (E[k][0] * v[0] + E[k][1] * v[1] + E[k][2] * v[2]);
}
double face_gsum(const nflbm_sim& s, int f, int u, int k) {
  const int (*E)[3] = s.lat == NFLBM_D2Q9 ? kD2Q9 : kD3Q19;
  const double* W = s.lat == NFLBM_D2Q9 ? kW2 : kW3;
  const double* v = s.face_v[f];
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double ev = E[k][0] * v[0] + E[k][1] * v[1] + E[k][2] * v[2];
  // s_k + s_kbar = 2 w_k (4.5 (e_k . v)^2 - 1.5 v.v)
  const double ssum = 2.0 * W[k] * (4.5 * ev * ev - 1.5 * vv);
  return s.face_c[f][u] * ssum - 2.0 * W[k] * s.m_geq * mu_bulk(s.co, s.face_c[f], s.omega, u);
}

// The device table of the open faces (internal component order).
template <class T>
void fill_faces(const nflbm_sim& s, FaceBC<T>* p) {
  std::memset(p, 0, sizeof(*p));
  p->open = s.open_mask | (s.out_face >= 0 ? 1 << s.out_face : 0);
  for (int f = 0; f < 6; ++f) {
    if (!((s.open_mask >> f) & 1)) continue;
    const double* Cu = s.face_c[f];
    for (int k = 1; k < s.Q; ++k) {
      p->fcorr[f][k] = static_cast<T>(face_fcorr(s, f, k));
      for (int i = 0; i < s.NE; ++i) p->gsum[f][i][k] = static_cast<T>(face_gsum(s, f, s.uidx[i], k));
    }
    for (int i = 0; i < s.N; ++i) p->cb[f][i] = static_cast<T>(Cu[s.uidx[i]]);
    p->eb[f] = static_cast<T>(bulk_energy_host(s.co, Cu));
  }
}

// Reconstruct C and evaluate the node fields of the current state.
int compute_fields(nflbm_sim* s) {
  int rc = ensure_fields(s);
  if (rc) return rc;
  StepArgs a = make_args(s, s->cur);
  HIPCHK(s, launch_conc(s->lat, s->N, s->store, conc_args(s, a), s->stream));
  HIPCHK(s, launch_update(s->lat, s->N, s->store, a, true, s->stream));
  return NFLBM_OK;
}


// Device arrays that make up the current state, in checkpoint order:
// f_1..f_{Q-1}, then the populations g_{i,0}, g_{i,k} (population form) or
// the node records C, mu~, (v, -3/2 v.v) (moment form).
std::vector<std::pair<void*, size_t>> state_segments(nflbm_sim* s) {
  const size_t n = s->n, Qm = s->Q - 1, NE = s->NE;
  std::vector<std::pair<void*, size_t>> v;
  // one segment per direction array: the checkpoint is packed, without the
  // gaps of the direction strides
  if (!s->fform)
    for (size_t k = 0; k < Qm; ++k)
      v.emplace_back(static_cast<unsigned char*>(s->f[s->cur]) + k * s->fstride * s->fs, n * s->fs);
  if (s->gform) {
    v.emplace_back(s->conc[s->cur], NE * n * s->ts);
    v.emplace_back(s->mu, NE * n * s->rs);
    v.emplace_back(s->vel, 4 * n * s->rs);
    if (s->fform) v.emplace_back(s->frec, 4 * n * s->rs);
  } else {
    v.emplace_back(s->g0[s->cur], NE * n * s->g0s);
    for (size_t k = 0; k < Qm; ++k)
      v.emplace_back(static_cast<unsigned char*>(s->gk[s->cur]) + k * s->gstride * s->fs, NE * n * s->fs);
  }
  if (s->out_face >= 0) v.emplace_back(s->out_buf, out_buf_bytes(s));
  return v;
}

// ------------------------------------------------------------ batches
int bfail(nflbm_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  else g_thread_error = msg;
  return code;
}

#define BHIPCHK(b, call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return bfail(b, NFLBM_EDEVICE, std::string(#call) + ": " + \
                                       hipGetErrorString(e_));                        \
  } while (0)

// Step arguments of member m under the batch launch shape, reading from
// population set src.
StepArgs batch_args(const nflbm_batch* b, const nflbm_sim* m, int src) {
  StepArgs a = make_args(m, src);
  const int TX = 1 << b->tx_log2, TY = 256 >> b->tx_log2;
  a.tx_log2 = b->tx_log2;
  a.tiles_x = (m->nx + TX - 1) / TX;
  a.tiles_y = (m->ny + TY - 1) / TY;
  return a;
}

void destroy_graphs(nflbm_batch* b) {
  for (int h = 0; h < 2; ++h) {
    if (b->exec[h]) (void)hipGraphExecDestroy(b->exec[h]);
    if (b->graph[h]) (void)hipGraphDestroy(b->graph[h]);
    b->exec[h] = nullptr;
    b->graph[h] = nullptr;
  }
}

void free_batch_tables(nflbm_batch* b) {
  if (b->args) (void)hipFree(b->args);
  if (b->work_conc) (void)hipFree(b->work_conc);
  if (b->work_update) (void)hipFree(b->work_update);
  b->args = nullptr;
  b->work_conc = b->work_update = nullptr;
}

// (Re)build the work lists and the step arguments of both parities for the
// members' current population sets.  Graph nodes keep pointing at the same
// buffers, so a captured graph stays valid as long as the lists keep their
// sizes; a new launch shape discards the graphs.
int build_batch_tables(nflbm_batch* b, bool new_shape) {
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  const int count = static_cast<int>(b->members.size());
  std::vector<int2> wc, wu;
  std::vector<StepArgs> args(2 * size_t(count));
  b->key.assign(count, 0);
  b->versions.assign(count, 0u);
  b->walls = 0;
  for (int i = 0; i < count; ++i) {
    const nflbm_sim* m = b->members[i];
    b->key[i] = m->cur;
    b->versions[i] = m->boundary_version;
    // one kernel variant for all members: the wall variant if any needs it
    if (m->wall[0] || m->wall[1] || m->wall[2] || m->bb) b->walls = 1;
    args[i] = batch_args(b, m, m->cur);
    args[count + i] = batch_args(b, m, m->cur ^ 1);
    for (StepArgs* x : {&args[i], &args[count + i]}) {
      x->nanflag = b->nanflag;
      x->flags |= kFlagCheckNaN;
    }
    const StepArgs& a = args[i];
    const long long nc = 1LL * a.tiles_x * a.tiles_y * m->nz;
    const long long nu = 1LL * a.tiles_x * a.tiles_y * a.chunks_z;
    if (static_cast<long long>(wc.size()) + nc > 0x7fffffffLL || static_cast<long long>(wu.size()) + nu > 0x7fffffffLL)
      return bfail(b, NFLBM_ENOTSUP, "batch too large: more than 2^31-1 workgroups per launch");
    for (long long t = 0; t < nc; ++t) wc.push_back(make_int2(i, static_cast<int>(t)));
    for (long long t = 0; t < nu; ++t) wu.push_back(make_int2(i, static_cast<int>(t)));
  }
  if (new_shape || !b->args || static_cast<int>(wc.size()) != b->blocks_conc ||
      static_cast<int>(wu.size()) != b->blocks_update) {
    destroy_graphs(b);
    free_batch_tables(b);
    bool ok = hipMalloc(reinterpret_cast<void**>(&b->args), args.size() * sizeof(StepArgs)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b->work_conc), wc.size() * sizeof(int2)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b->work_update), wu.size() * sizeof(int2)) == hipSuccess;
    if (!ok) {
      free_batch_tables(b);
      return bfail(b, NFLBM_ENOMEM, "cannot allocate the batch work lists");
    }
    b->blocks_conc = static_cast<int>(wc.size());
    b->blocks_update = static_cast<int>(wu.size());
  }
  BHIPCHK(b, hipMemcpyAsync(b->args, args.data(), args.size() * sizeof(StepArgs), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->work_conc, wc.data(), wc.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->work_update, wu.data(), wu.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  return NFLBM_OK;
}

// Which half of the argument table matches the members' current population
// sets (0 or 1); rebuilds the tables if some member was stepped on its own.
int batch_half(nflbm_batch* b, int* half) {
  const int count = static_cast<int>(b->members.size());
  bool same = true, flipped = true;
  for (int i = 0; i < count; ++i) {
    same = same && b->members[i]->cur == b->key[i];
    flipped = flipped && b->members[i]->cur != b->key[i];
  }
  if (same) { *half = 0; return NFLBM_OK; }
  if (flipped) { *half = 1; return NFLBM_OK; }
  *half = 0;
  return build_batch_tables(b, false);
}

bool batch_tile_fits(const nflbm_batch* b, int l) {
  const size_t lim = b->members[0]->lds_max;
  return update_lds_bytes(b->lat, b->N, b->store, l) <= lim &&
         (!b->members[0]->gform || conc_m_lds_bytes(b->lat, b->N, b->store, l, b->members[0]->fform) <= lim);
}

hipError_t launch_half(nflbm_batch* b, int half) {
  BatchLaunch bl{};
  bl.args = b->args + size_t(half) * b->members.size();
  bl.params = b->params;
  bl.work_conc = b->work_conc;
  bl.work_update = b->work_update;
  bl.blocks_conc = b->blocks_conc;
  bl.blocks_update = b->blocks_update;
  bl.tx_log2 = b->tx_log2;
  bl.walls = b->walls;
  bl.moments = b->members[0]->gform;
  bl.frecord = b->members[0]->fform;
  bool mob = false;
  for (const nflbm_sim* m : b->members) mob = mob || m->c2c2;
  hipError_t e = hipSuccess;
  if (!mob) {
    e = launch_batch_step(b->lat, b->N, b->store, bl, b->stream);
  } else {
    // members with the concentration-dependent mobility (Appendix C): their
    // potentials between the batch's reconstruction and update, their source
    // term after it, each on the member's arguments of this half
    bl.phase = 1;
    e = launch_batch_step(b->lat, b->N, b->store, bl, b->stream);
    for (size_t i = 0; i < b->members.size() && e == hipSuccess; ++i) {
      const nflbm_sim* m = b->members[i];
      if (m->c2c2)
        e = launch_mob_potentials(m->lat, m->N, m->store, mob_args(m, make_args(m, b->key[i] ^ half)), b->stream);
    }
    bl.phase = 2;
    if (e == hipSuccess) e = launch_batch_step(b->lat, b->N, b->store, bl, b->stream);
    for (size_t i = 0; i < b->members.size() && e == hipSuccess; ++i) {
      const nflbm_sim* m = b->members[i];
      if (m->c2c2)
        e = launch_mob_source(m->lat, m->N, m->store, mob_args(m, make_args(m, b->key[i] ^ half)), b->stream);
    }
  }
  // members with a convective outflow face: Eq. convect on the state this
  // half wrote (parity key ^ 1 after half 0, key after half 1)
  for (size_t i = 0; i < b->members.size() && e == hipSuccess; ++i) {
    const nflbm_sim* m = b->members[i];
    if (m->out_face < 0) continue;
    e = launch_outflow(m->lat, m->N, m->store, outflow_args(m, b->key[i] ^ (half == 0 ? 1 : 0), 0), b->stream);
  }
  return e;
}

// Capture graph_steps time steps of the whole batch, starting from argument
// half `half`, into an executable graph.
int capture_graph(nflbm_batch* b, int half) {
  hipGraph_t g = nullptr;
  BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int t = 0; t < b->graph_steps && e == hipSuccess; ++t) e = launch_half(b, (half + t) & 1);
  const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bfail(b, NFLBM_EDEVICE, std::string("graph capture failed: ") +
                                       hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return bfail(b, NFLBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  b->graph[half] = g;
  b->exec[half] = x;
  return NFLBM_OK;
}

int batch_run(nflbm_batch* b, long long nsteps, int mode) {
  if (mode == NFLBM_BATCH_PER_SIM) {
    for (nflbm_sim* m : b->members) {
      const int rc = nflbm_step(m, nsteps);
      if (rc != NFLBM_OK) return bfail(b, rc, m->err);
    }
    return NFLBM_OK;
  }
  BHIPCHK(b, nan_poll(&b->nan_pending, &b->nan_seen, b->nan_host, b->nan_ev, false));
  if (b->nan_seen) return bfail(b, NFLBM_ENUMERIC, "a NaN or Inf appeared in a member's state");
  for (size_t i = 0; i < b->members.size(); ++i) {
    if (i < b->versions.size() && b->members[i]->boundary_version == b->versions[i]) continue;
    // a member's solid nodes, open faces or outflow changed: new arguments,
    // and graphs that captured the old outflow launches are dropped
    destroy_graphs(b);
    const int rc = build_batch_tables(b, false);
    if (rc != NFLBM_OK) return rc;
    break;
  }
  bool local = false;
  for (nflbm_sim* m : b->members) local = local || m->f_local;
  if (local && nsteps > 0) {
    // record form of f: the first step after set_fields takes each node's
    // f from its own record (kFlagFLocal in those members' arguments); the
    // tables are then rebuilt without the flag for the remaining steps
    int rc = build_batch_tables(b, false);
    if (rc != NFLBM_OK) return rc;
    BHIPCHK(b, launch_half(b, 0));
    for (nflbm_sim* m : b->members) {
      m->cur ^= 1;
      m->f_local = false;
    }
    rc = build_batch_tables(b, false);
    if (rc != NFLBM_OK) return rc;
    if (nsteps == 1) {
      BHIPCHK(b, nan_enqueue(b->nanflag, b->nan_host, b->nan_ev, b->stream));
      b->nan_pending = true;
      return NFLBM_OK;
    }
    return batch_run(b, nsteps - 1, mode);
  }
  int half = 0;
  int rc = batch_half(b, &half);
  if (rc != NFLBM_OK) return rc;
  long long t = 0;
  if (mode == NFLBM_BATCH_GRAPH) {
    const long long reps = nsteps / b->graph_steps;
    if (reps > 0 && !b->exec[half]) {
      rc = capture_graph(b, half);
      if (rc != NFLBM_OK) return rc;
    }
    for (long long r = 0; r < reps; ++r) BHIPCHK(b, hipGraphLaunch(b->exec[half], b->stream));
    t = reps * b->graph_steps;  // an even count: the parity is unchanged
  }
  for (; t < nsteps; ++t) {
    BHIPCHK(b, launch_half(b, half));
    half ^= 1;
  }
  if (nsteps & 1)
    for (nflbm_sim* m : b->members) m->cur ^= 1;
  if (nsteps > 0) {
    BHIPCHK(b, nan_enqueue(b->nanflag, b->nan_host, b->nan_ev, b->stream));
    b->nan_pending = true;
  }
  return NFLBM_OK;
}

// Clear the batch's NaN flag (a member's state was set anew).
int batch_nan_reset(nflbm_batch* b) {
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  BHIPCHK(b, hipMemset(b->nanflag, 0, sizeof(int)));
  *b->nan_host = 0;
  b->nan_pending = false;
  b->nan_seen = 0;
  return NFLBM_OK;
}

// ------------------------------------------------------------ autotuning
std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::ostringstream o;
  o << prop.gcnArchName << "/cu" << prop.multiProcessorCount;
  std::string t = o.str();
  for (char& c : t)
    if (c == ' ' || c == '|') c = '_';
  return t;
}

// Cache file: one entry per line, "<key>|<values separated by spaces>"; the
// last line with a matching key wins.
bool cache_lookup(const char* path, const std::string& key, std::vector<int>* vals) {
  if (!path || !*path) return false;
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    const size_t bar = line.find('|');
    if (bar == std::string::npos || line.substr(0, bar) != key) continue;
    std::istringstream vs(line.substr(bar + 1));
    std::vector<int> v;
    int x;
    while (vs >> x) v.push_back(x);
    if (v.size() == vals->size()) {
      *vals = v;
      found = true;
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const std::vector<int>& vals) {
  if (!path || !*path) return;
  std::ofstream out(path, std::ios::app);
  if (!out) return;
  out << key << '|';
  for (size_t i = 0; i < vals.size(); ++i) out << (i ? " " : "") << vals[i];
  out << '\n';
}

std::string sim_key(const nflbm_sim* s) {
  std::ostringstream o;
  o << "sim lat=" << s->lat << " N=" << s->N << " store=" << s->store << " shape=" << s->nx << 'x' << s->ny
    << 'x' << s->nz << " walls=" << s->wall[0] << s->wall[1] << s->wall[2] << " solid=" << (s->bb ? 1 : 0) << " open=" << s->open_mask << " out=" << s->out_face
    << " flags=" << s->step_flags
    << " dev=" << device_tag();
  return o.str();
}

// Device copy of the current state of s (restored after timing).
struct SavedState {
  std::vector<void*> copies;
  int cur = 0;
  bool f_local = false;
};

int save_state(nflbm_sim* s, SavedState* st) {
  st->cur = s->cur;
  st->f_local = s->f_local;
  for (const auto& seg : state_segments(s)) {
    void* c = nullptr;
    if (hipMalloc(&c, seg.second) != hipSuccess) return fail(s, NFLBM_ENOMEM, "cannot allocate the autotuner's state copy");
    st->copies.push_back(c);
    HIPCHK(s, hipMemcpyAsync(c, seg.first, seg.second, hipMemcpyDeviceToDevice, s->stream));
  }
  return NFLBM_OK;
}

int restore_state(nflbm_sim* s, SavedState* st) {
  s->cur = st->cur;
  s->f_local = st->f_local;
  const auto segs = state_segments(s);
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < st->copies.size() && i < segs.size() && e == hipSuccess; ++i)
    e = hipMemcpyAsync(segs[i].first, st->copies[i], segs[i].second, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess && s->out_face >= 0 && s->gform)
    e = launch_outflow(s->lat, s->N, s->store, outflow_args(s, s->cur, 2), s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  for (void* c : st->copies) (void)hipFree(c);
  st->copies.clear();
  if (e != hipSuccess) return hip_fail(s, e, "autotune: restoring the state");
  return NFLBM_OK;
}

// Even number of timed steps giving roughly 5 ms of work per candidate.
long long tune_steps(double nodes, double bytes_per_node) {
  const double est = nodes * bytes_per_node / 4.0e12;  // seconds per step at 4 TB/s
  long long k = static_cast<long long>(5.0e-3 / (est > 0 ? est : 1e-6));
  if (k < 2) k = 2;
  if (k > 40) k = 40;
  return k & ~1LL;
}

// Validate cfg and fill every host-side field of s: sizes, coefficient
// tables, storage form of g, launch shape.  Allocates nothing.
int plan_sim(const nflbm_config* cfg, nflbm_sim* s) {
  if (cfg->lattice != NFLBM_D2Q9 && cfg->lattice != NFLBM_D3Q19)
    return fail(nullptr, NFLBM_EINVAL, "unknown lattice");
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)
    return fail(nullptr, NFLBM_EINVAL, "lattice dimensions must be >= 1");
  if (cfg->lattice == NFLBM_D2Q9 && cfg->nz != 1)
    return fail(nullptr, NFLBM_EINVAL, "D2Q9 needs nz == 1");
  const long long nn = 1LL * cfg->nx * cfg->ny * cfg->nz;
  if (nn >= (1LL << 31)) return fail(nullptr, NFLBM_EINVAL, "more than 2^31-1 nodes");
  const int N = cfg->ncomp;
  if (N < 2 || N > NFLBM_MAX_COMP) return fail(nullptr, NFLBM_EINVAL, "ncomp outside 2..8");
  if (!cfg->sigma || !cfg->tau) return fail(nullptr, NFLBM_EINVAL, "sigma and tau are required");
  if (cfg->precision < NFLBM_FP64 || cfg->precision > NFLBM_FP16S)
    return fail(nullptr, NFLBM_EINVAL, "unknown precision");
  const int imp = cfg->implicit_comp < 0 ? N - 1 : cfg->implicit_comp;
  if (imp >= N) return fail(nullptr, NFLBM_EINVAL, "implicit_comp out of range");
  for (int i = 0; i < N; ++i) {
    if (!(cfg->tau[i] > 0.5)) return fail(nullptr, NFLBM_EINVAL, "tau must exceed 1/2");
    if (cfg->tau_g && !(cfg->tau_g[i] > 0.5)) return fail(nullptr, NFLBM_EINVAL, "tau_g must exceed 1/2");
  }
  if (!(cfg->m > 0.0)) return fail(nullptr, NFLBM_EINVAL, "m must be positive");
  if (!(cfg->omega_stab >= 0.0)) return fail(nullptr, NFLBM_EINVAL, "omega_stab must be >= 0");
  for (int a = 0; a < 3; ++a)
    if (cfg->wall[a] != 0 && cfg->wall[a] != 1) return fail(nullptr, NFLBM_EINVAL, "wall flags are 0 or 1");
  if (cfg->lattice == NFLBM_D2Q9 && cfg->wall[2])
    return fail(nullptr, NFLBM_EINVAL, "D2Q9 has no z walls");

  s->lat = cfg->lattice;
  s->N = N;
  s->NE = N - 1;
  s->Q = s->lat == NFLBM_D2Q9 ? 9 : 19;
  s->store = cfg->precision;
  s->flags = cfg->flags;
  s->nx = cfg->nx;
  s->ny = cfg->ny;
  s->nz = cfg->nz;
  for (int a = 0; a < 3; ++a) s->wall[a] = cfg->wall[a];
  s->implicit = imp;
  s->n = static_cast<size_t>(nn);
  {
    int q = 0;
    for (int u = 0; u < N; ++u)
      if (u != imp) s->uidx[q++] = u;
    s->uidx[N - 1] = imp;
  }
  char msg[256] = {0};
  const int rc = compute_coeffs(N, cfg->sigma, cfg->width_D, &s->co, msg);
  if (rc) {
    return fail(nullptr, rc == -1 ? NFLBM_EINVAL : NFLBM_ESINGULAR, msg);
  }
  // Linear stability of the explicit Cahn-Hilliard update in a pure phase:
  // a mode of -lap eigenvalue lam grows by 1 + M lam (a - (3D/4) lam) per step
  // with a = -12/D; |growth| <= 1 up to lam_max = 16/3 needs the bound below.
  if (!(cfg->flags & (NFLBM_FLAG_ALLOW_UNSTABLE | NFLBM_FLAG_C2C2_MOBILITY))) {
    const double lam = 16.0 / 3.0;
    for (int i = 0; i < N; ++i) {
      const double tg = cfg->tau_g ? cfg->tau_g[i] : 1.0;
      const double M = cfg->m * (tg - 0.5) / 3.0;
      if (M * lam * (0.75 * cfg->width_D * lam + 12.0 / cfg->width_D) >= 2.0) {
            return fail(nullptr, NFLBM_EUNSTABLE,
                    "mobility M = c_s^2 m (tau_g - 1/2) exceeds the linear stability bound");
      }
    }
  }
  switch (s->store) {
    case NFLBM_FP64: s->fs = 8; s->g0s = 8; s->ts = 8; s->rs = 8; break;
    case NFLBM_FP32: s->fs = 4; s->g0s = 4; s->ts = 4; s->rs = 4; break;
    default: s->fs = 2; s->g0s = 4; s->ts = 4; s->rs = 2; break;
  }
  s->fstride = direction_stride(s->n, s->fs);
  s->gstride = direction_stride(s->n * size_t(s->NE), s->fs);
  s->step_flags = 0;
  for (int i = 0; i < N; ++i)
    if (cfg->tau_g && cfg->tau_g[i] != 1.0) s->step_flags |= kFlagNeedG;
  if (cfg->flags & NFLBM_FLAG_POTENTIAL_FORCE) s->step_flags |= kFlagPotential;
  if (cfg->flags & NFLBM_FLAG_NO_HYDRO) s->step_flags |= kFlagNoHydro;
  if (cfg->omega_stab != 0.0) s->step_flags |= kFlagOmega;
  // With every tau_g = 1 the post-collision g are equilibria of (C, mu~, v):
  // store those per node instead of the populations, unless asked not to.
  s->c2c2 = (cfg->flags & NFLBM_FLAG_C2C2_MOBILITY) != 0;
  s->gform = (!(s->step_flags & kFlagNeedG) && !(cfg->flags & NFLBM_FLAG_G_POPULATIONS) && !s->c2c2) ? 1 : 0;
  // With every node relaxing at omega+ = omega- = 1 (each tau_i = 1, BGK or
  // Lambda^TRT = 1/4) the post-collision f is fixed by the node's P, v and F
  // (Eqs. TRT, FTRT, hydroforce): keep those instead of the populations.
  bool unit = !(cfg->flags & NFLBM_FLAG_F_POPULATIONS) && !(cfg->flags & NFLBM_FLAG_NO_HYDRO);
  for (int i = 0; i < N && unit; ++i) {
    const double wp = 1.0 / cfg->tau[i];
    const double wm = cfg->trt_magic > 0.0 ? 1.0 / (0.5 + cfg->trt_magic / (cfg->tau[i] - 0.5)) : wp;
    unit = wp == 1.0 && wm == 1.0;
  }
  s->fform = (s->gform && unit) ? 1 : 0;
  if (s->gform && choose_launch(s) != 0) s->gform = s->fform = 0;   // its LDS window does not fit
  if (s->gform) s->step_flags |= kFlagMoments;
  if (s->fform) s->step_flags |= kFlagFRecord;
  if (choose_launch(s) != 0) {
    return fail(nullptr, NFLBM_ENOTSUP, "LDS window does not fit the device for this N and precision");
  }

  // Per-node arrays are addressed with 32-bit byte offsets from a uniform
  // base: the widest one must fit.  That is NE values a node (C, the g
  // populations of one direction, the rest populations), the four of the
  // moment form's velocity record, or the N flux potentials of the
  // concentration-dependent mobility.
  size_t width = s->NE;
  if (s->gform) width = std::max<size_t>(width, 4);
  if (s->c2c2) width = std::max<size_t>(width, size_t(s->N));
  const size_t vbytes = std::max(std::max(s->fs, s->ts), s->g0s);
  if (double(s->n) * double(width) * double(vbytes) >= 4294967296.0) {
    return fail(nullptr, NFLBM_ENOTSUP, "lattice too large: per-node byte offsets must fit 32 bits");
  }
  return NFLBM_OK;
}

// Device arrays of the state (pointer slot, bytes) in a fixed order: both f
// sets, then g (population form) or the node records (moment form), then
// the reconstructed C and E_B.
std::vector<std::pair<void**, size_t>> state_arrays(nflbm_sim* s) {
  const size_t n = s->n, Qm = s->Q - 1, NE = s->NE;
  std::vector<std::pair<void**, size_t>> v;
  if (!s->fform)
    for (int b = 0; b < 2; ++b) v.emplace_back(&s->f[b], Qm * s->fstride * s->fs);
  if (s->gform) {
    for (int b = 0; b < 2; ++b) v.emplace_back(&s->conc[b], NE * n * s->ts);
    v.emplace_back(&s->mu, NE * n * s->rs);
    v.emplace_back(&s->vel, 4 * n * s->rs);
    if (s->fform) {
      v.emplace_back(&s->frec, 4 * n * s->rs);
      v.emplace_back(&s->fmom, 4 * n * s->rs);
    }
  } else {
    for (int b = 0; b < 2; ++b) v.emplace_back(&s->g0[b], NE * n * s->g0s);
    for (int b = 0; b < 2; ++b) v.emplace_back(&s->gk[b], Qm * s->gstride * s->fs);
    v.emplace_back(&s->conc[0], NE * n * s->ts);
  }
  v.emplace_back(&s->eb, n * s->ts);
  return v;
}

// The device table of the open and outflow faces (freed when there is none).
int upload_faces(nflbm_sim* sim) {
  if (!sim->open_mask && sim->out_face < 0) {
    if (sim->faces) (void)hipFree(sim->faces);
    sim->faces = nullptr;
    return NFLBM_OK;
  }
  const size_t bytes = sim->ts == 8 ? sizeof(FaceBC<double>) : sizeof(FaceBC<float>);
  if (!sim->faces && hipMalloc(&sim->faces, bytes) != hipSuccess) {
    sim->faces = nullptr;
    return fail(sim, NFLBM_ENOMEM, "cannot allocate the open-face table");
  }
  hipError_t e;
  if (sim->ts == 8) {
    auto* t = new FaceBC<double>();
    fill_faces(*sim, t);
    e = hipMemcpy(sim->faces, t, sizeof(*t), hipMemcpyHostToDevice);
    delete t;
  } else {
    auto* t = new FaceBC<float>();
    fill_faces(*sim, t);
    e = hipMemcpy(sim->faces, t, sizeof(*t), hipMemcpyHostToDevice);
    delete t;
  }
  if (e != hipSuccess) return hip_fail(sim, e, "set_open_face");
  return NFLBM_OK;
}

constexpr size_t kBindAlign = 256;
size_t align_up(size_t v) { return (v + kBindAlign - 1) / kBindAlign * kBindAlign; }

}  // namespace

namespace nflbm {

int sim_device(const nflbm_sim* s) { return s->device; }

int sim_fail(nflbm_sim* s, int code, const char* msg) { return fail(s, code, msg); }

int diag_run(nflbm_sim* sim, int vcm_component, double* partial, int max_blocks, double* result, nflbm_diag* out) {
  if (!sim || !out) return fail(sim, NFLBM_EINVAL, "NULL argument");
  if (vcm_component < 0 || vcm_component >= sim->N) return fail(sim, NFLBM_EINVAL, "vcm_component out of range");
  const int N = sim->N;
  const int rec = reduce_record_len(N);
  StepArgs a = make_args(sim, sim->cur);
  HIPCHK(sim, launch_conc(sim->lat, N, sim->store, conc_args(sim, a), sim->stream));
  a.diag_partial = partial;
  for (int i = 0; i < N; ++i)
    if (sim->uidx[i] == vcm_component) a.diag_vcm = i;
  int blocks = 0;
  HIPCHK(sim, launch_diag(sim->lat, N, sim->store, a, max_blocks, result, &blocks, sim->stream));
  double r[3 * kMaxComp + 9];
  HIPCHK(sim, hipMemcpyAsync(r, result, rec * sizeof(double), hipMemcpyDeviceToHost, sim->stream));
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  std::memset(out, 0, sizeof(*out));
  for (int i = 0; i < N; ++i) {   // the record is in internal component order
    const int u = sim->uidx[i];
    out->mass[u] = r[i];
    out->max_abs_c[u] = r[N + 3 + i];
    out->min_c[u] = r[2 * N + 3 + i];
  }
  for (int d = 0; d < 3; ++d) out->momentum[d] = r[N + d];
  out->max_sum_dev = r[3 * N + 3];
  const double cm = r[3 * N + 7];
  for (int d = 0; d < 3; ++d) out->vcm[d] = cm != 0.0 ? r[3 * N + 4 + d] / cm : 0.0;
  out->vcm_component = vcm_component;
  out->nan = r[3 * N + 8] != 0.0 ? 1 : 0;
  if (out->nan) return fail(sim, NFLBM_ENUMERIC, "NaN or Inf in the state");
  return NFLBM_OK;
}

}  // namespace nflbm

extern "C" {

int nflbm_abi_version(void) { return NFLBM_ABI_VERSION; }

const char* nflbm_last_error(const nflbm_sim* sim) {
  return sim ? sim->err.c_str() : g_thread_error.c_str();
}

int nflbm_coefficients(int N, const double* sigma, double D, double* alpha, double* gamma,
                       double* psi, double* xtab, double* ztab) {
  if (!sigma) return fail(nullptr, NFLBM_EINVAL, "sigma is NULL");
  Coeffs c;
  char msg[256] = {0};
  const int rc = compute_coeffs(N, sigma, D, &c, msg);
  if (rc == -1) return fail(nullptr, NFLBM_EINVAL, msg);
  if (rc == -2) return fail(nullptr, NFLBM_ESINGULAR, msg);
  for (int i = 0; i < N; ++i) {
    if (gamma) gamma[i] = c.gamma[i];
    for (int j = 0; j < N; ++j) {
      if (alpha) alpha[i * N + j] = c.alpha[i][j];
      for (int k = 0; k < N; ++k) {
        const size_t o = (size_t(i) * N + j) * N + k;
        if (psi) psi[o] = c.psi[i][j][k];
        if (xtab) xtab[o] = c.xt[i][j][k];
        if (ztab) ztab[o] = c.zt[i][j][k];
      }
    }
  }
  return NFLBM_OK;
}

int nflbm_create(const nflbm_config* cfg, nflbm_sim** out) {
  if (!cfg || !out) return fail(nullptr, NFLBM_EINVAL, "NULL argument");
  *out = nullptr;
  nflbm_sim* s = new nflbm_sim();
  const int prc = plan_sim(cfg, s);
  if (prc != NFLBM_OK) {
    delete s;
    return prc;
  }
  const int N = s->N;
  const size_t n = s->n;
  bool ok = hipGetDevice(&s->device) == hipSuccess;
  for (auto& a : state_arrays(s)) ok = ok && hipMalloc(a.first, a.second) == hipSuccess;
  const size_t psize = s->ts == 8 ? sizeof(DevParams<double>) : sizeof(DevParams<float>);
  ok = ok && hipMalloc(&s->params, psize) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&s->nanflag), sizeof(int)) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&s->nan_host), sizeof(int), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&s->nan_ev, hipEventDisableTiming) == hipSuccess;
  if (s->c2c2) {
    const size_t msize = s->ts == 8 ? sizeof(MobParams<double>) : sizeof(MobParams<float>);
    ok = ok && hipMalloc(&s->mob, msize) == hipSuccess;
    ok = ok && hipMalloc(&s->phi, size_t(N) * n * s->ts) == hipSuccess;
  }
  if (!ok) {
    free_device(s);
    delete s;
    return fail(nullptr, NFLBM_ENOMEM, "device allocation failed");
  }
  // the concentration-dependent mobility takes m = 0 in g^eq; cfg->m is its m*
  const double m_geq = s->c2c2 ? 0.0 : cfg->m;
  s->m_geq = m_geq;
  s->omega = cfg->omega_stab;
  if (s->ts == 8) {
    DevParams<double> p;
    fill_params(*s, cfg->tau, cfg->tau_g, cfg->trt_magic, m_geq, cfg->omega_stab, cfg->body_force, &p);
    if (hipMemcpy(s->params, &p, sizeof(p), hipMemcpyHostToDevice) != hipSuccess) ok = false;
  } else {
    DevParams<float> p;
    fill_params(*s, cfg->tau, cfg->tau_g, cfg->trt_magic, m_geq, cfg->omega_stab, cfg->body_force, &p);
    if (hipMemcpy(s->params, &p, sizeof(p), hipMemcpyHostToDevice) != hipSuccess) ok = false;
  }
  if (ok && s->c2c2) {
    if (s->ts == 8) {
      auto* mp = new MobParams<double>();
      fill_mob(*s, cfg->tau_g, cfg->m, mp);
      if (hipMemcpy(s->mob, mp, sizeof(*mp), hipMemcpyHostToDevice) != hipSuccess) ok = false;
      delete mp;
    } else {
      auto* mp = new MobParams<float>();
      fill_mob(*s, cfg->tau_g, cfg->m, mp);
      if (hipMemcpy(s->mob, mp, sizeof(*mp), hipMemcpyHostToDevice) != hipSuccess) ok = false;
      delete mp;
    }
  }
  // rest state with C_1 = 1 everywhere until set_fields is called
  if (ok) {
    std::vector<double> C(size_t(N) * n, 0.0);
    for (size_t q = 0; q < n; ++q) C[q] = 1.0;
    *out = s;
    const int r2 = nflbm_set_fields(s, C.data(), nullptr, nullptr);
    if (r2 != NFLBM_OK) {
      std::string m2 = s->err;
      free_device(s);
      delete s;
      *out = nullptr;
      return fail(nullptr, r2, m2);
    }
    return NFLBM_OK;
  }
  free_device(s);
  delete s;
  return fail(nullptr, NFLBM_EDEVICE, "cannot upload parameters");
}

void nflbm_destroy(nflbm_sim* sim) {
  if (!sim) return;
  if (sim->stream) (void)hipStreamSynchronize(sim->stream);
  else (void)hipDeviceSynchronize();
  free_device(sim);
  delete sim;
}

int nflbm_set_stream(nflbm_sim* sim, void* stream) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  sim->stream = static_cast<hipStream_t>(stream);
  return NFLBM_OK;
}

// Whether the open faces (mask), the outflow face (-1: none) and the solid
// mask (empty: none) can go together: solid nodes continue straight through
// the outflow plane (the same on planes N and N-1), and an open face on
// another axis meets the outflow plane only at solid nodes (so no fluid node
// mixes the outflow with another open face).  On success *fluid is the
// number of fluid nodes on plane N-1 (0 without an outflow face).
static int check_boundaries(nflbm_sim* sim, int open_mask, int out_face, const unsigned char* solid,
                            double* fluid) {
  *fluid = 0.0;
  if (out_face < 0) return NFLBM_OK;
  const int dims[3] = {sim->nx, sim->ny, sim->nz};
  const int ax = out_face / 2;
  const int t0 = ax == 0 ? 1 : 0, t1 = ax == 2 ? 1 : 2;
  const int pN = (out_face & 1) ? dims[ax] - 1 : 0;
  const int pI = (out_face & 1) ? dims[ax] - 2 : 1;
  auto at = [&](int a, int b, int c) {   // node of (axis ax = a, t0 = b, t1 = c)
    int xyz[3];
    xyz[ax] = a;
    xyz[t0] = b;
    xyz[t1] = c;
    return size_t(xyz[0]) + size_t(sim->nx) * (size_t(xyz[1]) + size_t(sim->ny) * size_t(xyz[2]));
  };
  size_t cnt = 0;
  for (int c = 0; c < dims[t1]; ++c)
    for (int b = 0; b < dims[t0]; ++b) {
      const bool sN = solid && solid[at(pN, b, c)];
      const bool sI = solid && solid[at(pI, b, c)];
      if (sN != sI)
        return fail(sim, NFLBM_ENOTSUP,
                    "solid nodes must continue straight through the outflow plane (the same on it and the plane inside it)");
      if (!sI) ++cnt;
      // an open face of another axis touching this plane node
      for (int f = 0; f < 6; ++f) {
        if (!((open_mask >> f) & 1) || f / 2 == ax) continue;
        const int fa = f / 2;
        const int pos = (f & 1) ? dims[fa] - 1 : 0;
        const int coord = fa == t0 ? b : c;
        if (coord == pos && !sN)
          return fail(sim, NFLBM_ENOTSUP,
                      "an open face on another axis may meet the outflow face only at solid nodes");
      }
    }
  if (cnt == 0) return fail(sim, NFLBM_EINVAL, "no fluid node on the plane inside the outflow face");
  *fluid = double(cnt);
  return NFLBM_OK;
}

int nflbm_set_open_face(nflbm_sim* sim, int face, const double* v_b, const double* C_b) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  if (face < 0 || face >= 6 || (sim->lat == NFLBM_D2Q9 && face >= 4))
    return fail(sim, NFLBM_EINVAL, "face is 0..5 (x-, x+, y-, y+, z-, z+; 0..3 in D2Q9)");
  if (!sim->wall[face / 2]) return fail(sim, NFLBM_EINVAL, "an open face must lie on a walled axis");
  if (sim->c2c2) return fail(sim, NFLBM_ENOTSUP, "open faces take no concentration-dependent mobility");
  if ((v_b == nullptr) != (C_b == nullptr)) return fail(sim, NFLBM_EINVAL, "v_b and C_b go together");
  if (v_b && face == sim->out_face) return fail(sim, NFLBM_EINVAL, "the face is the outflow face");
  if (v_b) {
    double fluid = 0.0;
    const int rc = check_boundaries(sim, sim->open_mask | (1 << face), sim->out_face,
                                    sim->solid_host.empty() ? nullptr : sim->solid_host.data(), &fluid);
    if (rc) return rc;
  }
  if (v_b) {
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(v_b[d])) return fail(sim, NFLBM_EINVAL, "v_b must be finite");
    double sum = 0.0;
    for (int i = 0; i < sim->N; ++i) {
      if (!std::isfinite(C_b[i])) return fail(sim, NFLBM_EINVAL, "C_b must be finite");
      sum += C_b[i];
    }
    if (std::fabs(sum - 1.0) > 1e-12) return fail(sim, NFLBM_EINVAL, "C_b must sum to 1");
    for (int d = 0; d < 3; ++d) sim->face_v[face][d] = v_b[d];
    for (int i = 0; i < sim->N; ++i) sim->face_c[face][i] = C_b[i];
    sim->open_mask |= 1 << face;
  } else {
    sim->open_mask &= ~(1 << face);
  }
  ++sim->boundary_version;
  return upload_faces(sim);
}

int nflbm_set_outflow(nflbm_sim* sim, int face) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  if (face == -1) {
    if (sim->out_face < 0) return NFLBM_OK;
    sim->out_face = -1;
    ++sim->boundary_version;
    if (sim->out_buf) (void)hipFree(sim->out_buf);
    if (sim->out_red) (void)hipFree(sim->out_red);
    sim->out_buf = nullptr;
    sim->out_red = nullptr;
    return upload_faces(sim);
  }
  if (face < 0 || face >= 6 || (sim->lat == NFLBM_D2Q9 && face >= 4))
    return fail(sim, NFLBM_EINVAL, "face is 0..5 (x-, x+, y-, y+, z-, z+; 0..3 in D2Q9), or -1");
  const int dims[3] = {sim->nx, sim->ny, sim->nz};
  if (!sim->wall[face / 2]) return fail(sim, NFLBM_EINVAL, "an outflow face must lie on a walled axis");
  if (dims[face / 2] < 3) return fail(sim, NFLBM_EINVAL, "the outflow axis needs at least 3 nodes");
  if ((sim->open_mask >> face) & 1) return fail(sim, NFLBM_EINVAL, "the face is an open face");
  if (sim->c2c2) return fail(sim, NFLBM_ENOTSUP, "an outflow face takes no concentration-dependent mobility");
  double fluid = 0.0;
  {
    const int rc = check_boundaries(sim, sim->open_mask, face,
                                    sim->solid_host.empty() ? nullptr : sim->solid_host.data(), &fluid);
    if (rc) return rc;
  }
  if (sim->out_face >= 0 && sim->out_face != face) {
    const int rc = nflbm_set_outflow(sim, -1);
    if (rc) return rc;
  }
  const int ax = face / 2;
  const size_t P = size_t(dims[ax == 0 ? 1 : 0]) * size_t(dims[ax == 2 ? 1 : 2]);
  if (!sim->out_buf) {
    sim->out_plane = P;
    sim->out_face = face;   // sizes the buffer
    const long long blocks = static_cast<long long>((P + kOutNodes - 1) / kOutNodes);
    if (blocks > (1LL << 30)) {
      sim->out_face = -1;
      return fail(sim, NFLBM_EINVAL, "outflow plane too large");
    }
    sim->out_blocks = static_cast<int>(blocks);
    if (hipMalloc(&sim->out_buf, out_buf_bytes(sim)) != hipSuccess) {
      sim->out_buf = nullptr;
      sim->out_face = -1;
      return fail(sim, NFLBM_ENOMEM, "cannot allocate the outflow plane buffers");
    }
    if (hipMalloc(reinterpret_cast<void**>(&sim->out_red), size_t(sim->out_blocks + 1) * sizeof(double)) !=
        hipSuccess) {
      (void)hipFree(sim->out_buf);
      sim->out_buf = nullptr;
      sim->out_red = nullptr;
      sim->out_face = -1;
      return fail(sim, NFLBM_ENOMEM, "cannot allocate the outflow reduction buffer");
    }
  }
  sim->out_face = face;
  sim->out_fluid = fluid;
  ++sim->boundary_version;
  int rc = upload_faces(sim);
  if (rc) return rc;
  // start from the current state's boundary plane
  rc = launch_outflow_step(sim, 1);
  if (rc) return rc;
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  return NFLBM_OK;
}

int nflbm_set_solid(nflbm_sim* sim, const unsigned char* solid) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  double fluid_out = 0.0;
  {
    const int rc = check_boundaries(sim, sim->open_mask, sim->out_face, solid, &fluid_out);
    if (rc) return rc;
  }
  if (!solid) {
    if (sim->bb) (void)hipFree(sim->bb);
    sim->bb = nullptr;
    sim->solid_host.clear();
    sim->out_fluid = fluid_out;
    if (!sim->shape_chosen) (void)default_launch(sim);
    ++sim->boundary_version;
    return NFLBM_OK;
  }
  const size_t n = sim->n;
  size_t fluid = 0;
  for (size_t q = 0; q < n; ++q) fluid += solid[q] ? 0 : 1;
  if (fluid == 0) return fail(sim, NFLBM_EINVAL, "every node is solid");
  if (!sim->bb && hipMalloc(reinterpret_cast<void**>(&sim->bb), n * sizeof(uint32_t)) != hipSuccess) {
    sim->bb = nullptr;
    return fail(sim, NFLBM_ENOMEM, "cannot allocate the solid geometry");
  }
  unsigned char* dmask = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&dmask), n) != hipSuccess)
    return fail(sim, NFLBM_ENOMEM, "cannot allocate the solid mask");
  hipError_t e = hipMemcpyAsync(dmask, solid, n, hipMemcpyHostToDevice, sim->stream);
  if (e == hipSuccess) e = launch_build_bb(sim->lat, dmask, sim->bb, make_args(sim, sim->cur), sim->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
  (void)hipFree(dmask);
  if (e != hipSuccess) return hip_fail(sim, e, "set_solid");
  sim->solid_host.assign(solid, solid + n);
  sim->out_fluid = fluid_out;
  {
    const int rc = refresh_outflow_plane(sim);
    if (rc) return rc;
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
  }
  // the default launch shape depends on whether solid nodes are present
  if (!sim->shape_chosen) (void)default_launch(sim);
  ++sim->boundary_version;
  return NFLBM_OK;
}

int nflbm_set_fields(nflbm_sim* sim, const double* C, const double* v, const double* P) {
  if (!sim || !C) return fail(sim, NFLBM_EINVAL, "NULL argument");
  const size_t n = sim->n;
  // A uniform pressure adds 3 w_k P_ref to every f_k (Eq. feq, pressure
  // form), a shift that streaming, both collisions, bounce-back, the open
  // faces and the outflow all map onto itself: the state keeps P - P_ref,
  // whose populations stay small (binary16 storage keeps its precision).
  std::vector<double> Pshift;
  sim->p_ref = 0.0;
  if (P) {
    double sum = 0.0, lo = 0.0, hi = 0.0;
    size_t cnt = 0;
    for (size_t q = 0; q < n; ++q) {
      if (!sim->solid_host.empty() && sim->solid_host[q]) continue;
      lo = cnt ? std::min(lo, P[q]) : P[q];
      hi = cnt ? std::max(hi, P[q]) : P[q];
      sum += P[q];
      ++cnt;
    }
    // a uniform P is taken exactly (its summed mean can be off by rounding)
    sim->p_ref = !cnt ? 0.0 : (lo == hi ? lo : sum / double(cnt));
    if (!std::isfinite(sim->p_ref)) sim->p_ref = 0.0;   // a NaN in P stays in the state
    Pshift.assign(P, P + n);
    for (double& x : Pshift) x -= sim->p_ref;
    P = Pshift.data();
  }
  const size_t cnt = size_t(sim->N) * n + (v ? 3 * n : 0) + (P ? n : 0);
  double* tmp = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&tmp), cnt * sizeof(double)) != hipSuccess)
    return fail(sim, NFLBM_ENOMEM, "cannot allocate the initialisation buffer");
  double* dC = tmp;
  double* dv = v ? tmp + size_t(sim->N) * n : nullptr;
  double* dP = P ? tmp + size_t(sim->N) * n + (v ? 3 * n : 0) : nullptr;
  hipError_t e = hipMemcpyAsync(dC, C, size_t(sim->N) * n * sizeof(double), hipMemcpyHostToDevice, sim->stream);
  if (e == hipSuccess && v) e = hipMemcpyAsync(dv, v, 3 * n * sizeof(double), hipMemcpyHostToDevice, sim->stream);
  if (e == hipSuccess && P) e = hipMemcpyAsync(dP, P, n * sizeof(double), hipMemcpyHostToDevice, sim->stream);
  if (e == hipSuccess) {
    InitArgs a{};
    a.f = sim->f[sim->cur];
    a.g0 = sim->g0[sim->cur];   // population form (null in the moment form, whose
    a.gk = sim->gk[sim->cur];   // records are reached through a.sa)
    a.C = dC;
    a.v = dv;
    a.P = dP;
    a.params = sim->params;
    a.n = static_cast<long long>(n);
    a.sa = make_args(sim, sim->cur);
    e = launch_init(sim->lat, sim->N, sim->store, a, sim->stream);
  }
  if (e == hipSuccess && (sim->step_flags & kFlagNoHydro))
    // f is never written in diffusive-only runs: both sets hold the initial f
    e = hipMemcpyAsync(sim->f[1 - sim->cur], sim->f[sim->cur], size_t(sim->Q - 1) * sim->fstride * sim->fs,
                       hipMemcpyDeviceToDevice, sim->stream);
  if (e == hipSuccess && sim->out_face >= 0) {
    // the outflow plane and ghosts start from the new state
    const int rc = launch_outflow_step(sim, 1);
    if (rc) {
      (void)hipStreamSynchronize(sim->stream);
      (void)hipFree(tmp);
      return rc;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(sim, e, "set_fields");
  // moment form: the first step starts from the initial populations (the
  // record form of f takes each node's f as the equilibrium of its own
  // record, which the population form stores at every node; g entering
  // across an open face is the initial 0)
  sim->f_local = sim->gform != 0;
  return sim_nan_reset(sim);
}

int nflbm_step(nflbm_sim* sim, long long nsteps) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  if (nsteps < 0) return fail(sim, NFLBM_EINVAL, "nsteps < 0");
  // a NaN reported by the copy behind an earlier call
  int rc = sim_nan_status(sim, false);
  if (rc != NFLBM_OK) return rc;
  bool checked = false;
  for (long long t = 0; t < nsteps; ++t) {
    rc = launch_step(sim, nullptr, nullptr, &checked);
    if (rc != NFLBM_OK) return rc;
  }
  if (checked) {
    // the device flag only ever goes from 0 to 1, so a newer copy subsumes
    // one still in flight; the event follows the newest
    HIPCHK(sim, nan_enqueue(sim->nanflag, sim->nan_host, sim->nan_ev, sim->stream));
    sim->nan_pending = true;
  }
  return NFLBM_OK;
}

int nflbm_synchronize(nflbm_sim* sim) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  HIPCHK(sim, nan_poll(&sim->nan_pending, &sim->nan_seen, sim->nan_host, sim->nan_ev, true));
  // the flag as the last checked step left it
  HIPCHK(sim, hipMemcpy(sim->nan_host, sim->nanflag, sizeof(int), hipMemcpyDeviceToHost));
  if (*sim->nan_host) sim->nan_seen = 1;
  return sim_nan_status(sim, true);
}

int nflbm_set_nan_check(nflbm_sim* sim, long long every) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  if (every < 0) return fail(sim, NFLBM_EINVAL, "every must be >= 0");
  sim->nan_every = every;
  return NFLBM_OK;
}

int nflbm_step_timed(nflbm_sim* sim, long long nsteps, double* ms, double* ms_update) {
  if (!sim || !ms) return fail(sim, NFLBM_EINVAL, "NULL argument");
  hipEvent_t e0, e1;
  HIPCHK(sim, hipEventCreate(&e0));
  HIPCHK(sim, hipEventCreate(&e1));
  std::vector<hipEvent_t> ev;
  if (ms_update) {
    ev.resize(2 * size_t(nsteps));
    for (auto& x : ev) HIPCHK(sim, hipEventCreate(&x));
  }
  int rc0 = sim_nan_status(sim, true);
  if (rc0 != NFLBM_OK) return rc0;
  bool checked = false;
  HIPCHK(sim, hipEventRecord(e0, sim->stream));
  for (long long t = 0; t < nsteps; ++t) {
    const int rc = ms_update ? launch_step(sim, ev[2 * t], ev[2 * t + 1], &checked)
                             : launch_step(sim, nullptr, nullptr, &checked);
    if (rc != NFLBM_OK) return rc;
  }
  HIPCHK(sim, hipEventRecord(e1, sim->stream));
  if (checked) {
    HIPCHK(sim, nan_enqueue(sim->nanflag, sim->nan_host, sim->nan_ev, sim->stream));
    sim->nan_pending = true;
  }
  HIPCHK(sim, hipEventSynchronize(e1));
  float t_ms = 0.f;
  HIPCHK(sim, hipEventElapsedTime(&t_ms, e0, e1));
  *ms = t_ms;
  if (ms_update) {
    double tot = 0.0;
    for (long long t = 0; t < nsteps; ++t) {
      float u = 0.f;
      HIPCHK(sim, hipEventElapsedTime(&u, ev[2 * t], ev[2 * t + 1]));
      tot += u;
    }
    *ms_update = tot;
    for (auto& x : ev) (void)hipEventDestroy(x);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return sim_nan_status(sim, true);
}

int nflbm_step_timed_kernels(nflbm_sim* sim, long long nsteps, double* ms_conc, double* ms_update) {
  if (!sim || !ms_conc || !ms_update) return fail(sim, NFLBM_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(sim, NFLBM_EINVAL, "nsteps < 0");
  int rc = sim_nan_status(sim, true);
  if (rc != NFLBM_OK) return rc;
  std::vector<hipEvent_t> ev(4 * size_t(nsteps));
  for (auto& x : ev) HIPCHK(sim, hipEventCreate(&x));
  bool checked = false;
  for (long long t = 0; t < nsteps; ++t) {
    rc = launch_step(sim, ev[4 * t + 2], ev[4 * t + 3], &checked, ev[4 * t], ev[4 * t + 1]);
    if (rc != NFLBM_OK) return rc;
  }
  if (checked) {
    HIPCHK(sim, nan_enqueue(sim->nanflag, sim->nan_host, sim->nan_ev, sim->stream));
    sim->nan_pending = true;
  }
  if (nsteps > 0) HIPCHK(sim, hipEventSynchronize(ev.back()));
  double tc = 0.0, tu = 0.0;
  for (long long t = 0; t < nsteps; ++t) {
    float a = 0.f, b = 0.f;
    HIPCHK(sim, hipEventElapsedTime(&a, ev[4 * t], ev[4 * t + 1]));
    HIPCHK(sim, hipEventElapsedTime(&b, ev[4 * t + 2], ev[4 * t + 3]));
    tc += a;
    tu += b;
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  *ms_conc = tc;
  *ms_update = tu;
  return sim_nan_status(sim, true);
}

int nflbm_get_field(nflbm_sim* sim, int field, double* host_out) {
  if (!sim || !host_out) return fail(sim, NFLBM_EINVAL, "NULL argument");
  const size_t n = sim->n;
  const int N = sim->N;
  if (field >= NFLBM_FIELD_C && field <= NFLBM_FIELD_MU) {
    int rc = compute_fields(sim);
    if (rc) return rc;
    size_t off = 0, cnt = 0;
    switch (field) {
      case NFLBM_FIELD_C: off = 0; cnt = N; break;
      case NFLBM_FIELD_V: off = N; cnt = 3; break;
      case NFLBM_FIELD_P: off = N + 3; cnt = 1; break;
      case NFLBM_FIELD_F: off = N + 4; cnt = 3; break;
      default: off = N + 7; cnt = N; break;
    }
    HIPCHK(sim, hipMemcpyAsync(host_out, sim->fields + off * n, cnt * n * sizeof(double),
                               hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    if (field == NFLBM_FIELD_P && sim->p_ref != 0.0)
      for (size_t q = 0; q < n; ++q)
        if (sim->solid_host.empty() || !sim->solid_host[q]) host_out[q] += sim->p_ref;
    return NFLBM_OK;
  }
  if (field == NFLBM_FIELD_F_RAW || field == NFLBM_FIELD_G_RAW) {
    // The device holds post-collision populations (pull streaming); the
    // post-streaming values are gathered here on the host.
    const int Qm = sim->Q - 1;
    const int NE = sim->NE;
    std::vector<unsigned char> fbuf, g0buf, gkbuf;
    const size_t fst = sim->fstride, gst = sim->gstride;
    // bytes of a stored f value (the record form writes them out in the
    // compute precision)
    const size_t fbytes = sim->fform ? sim->ts : sim->fs;
    if (field == NFLBM_FIELD_F_RAW && sim->fform) {
      fbuf.resize(Qm * fst * sim->ts);
      void* tmp = nullptr;
      if (hipMalloc(&tmp, fbuf.size()) != hipSuccess)
        return fail(sim, NFLBM_ENOMEM, "cannot allocate the population read-back buffer");
      hipError_t e = launch_expand_f(sim->lat, sim->store, make_args(sim, sim->cur), tmp, sim->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(fbuf.data(), tmp, fbuf.size(), hipMemcpyDeviceToHost, sim->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
      (void)hipFree(tmp);
      if (e != hipSuccess) return hip_fail(sim, e, "F_RAW read-back");
    } else if (field == NFLBM_FIELD_F_RAW) {
      fbuf.resize(Qm * fst * sim->fs);
      HIPCHK(sim, hipMemcpyAsync(fbuf.data(), sim->f[sim->cur], fbuf.size(), hipMemcpyDeviceToHost, sim->stream));
    } else {
      g0buf.resize(size_t(NE) * n * sim->g0s);
      gkbuf.resize(Qm * gst * sim->fs);
      const void* g0dev = sim->g0[sim->cur];
      const void* gkdev = sim->gk[sim->cur];
      void* tmp = nullptr;
      if (sim->gform) {
        // the moment form holds no populations: write them out from the
        // node records, as the population form would have stored them
        if (hipMalloc(&tmp, g0buf.size() + gkbuf.size()) != hipSuccess)
          return fail(sim, NFLBM_ENOMEM, "cannot allocate the population read-back buffer");
        StepArgs a = make_args(sim, sim->cur);
        a.g0_dst = tmp;
        a.gk_dst = static_cast<unsigned char*>(tmp) + g0buf.size();
        const hipError_t e = launch_expand(sim->lat, sim->N, sim->store, a, sim->stream);
        if (e != hipSuccess) {
          (void)hipFree(tmp);
          return hip_fail(sim, e, "launch_expand");
        }
        g0dev = a.g0_dst;
        gkdev = a.gk_dst;
      }
      hipError_t e = hipMemcpyAsync(g0buf.data(), g0dev, g0buf.size(), hipMemcpyDeviceToHost, sim->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(gkbuf.data(), gkdev, gkbuf.size(), hipMemcpyDeviceToHost, sim->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
      if (tmp) (void)hipFree(tmp);
      if (e != hipSuccess) return hip_fail(sim, e, "G_RAW read-back");
    }
    HIPCHK(sim, hipStreamSynchronize(sim->stream));
    auto val = [&](const unsigned char* base, size_t idx, size_t bytes, bool moving) -> double {
      if (bytes == 8) return reinterpret_cast<const double*>(base)[idx];
      if (bytes == 4) return reinterpret_cast<const float*>(base)[idx];
      const _Float16 h = reinterpret_cast<const _Float16*>(base)[idx];
      return moving ? static_cast<double>(static_cast<float>(h) * (1.0f / kHalfScale)) : 0.0;
    };
    const int (*E)[3] = sim->lat == NFLBM_D2Q9 ? kD2Q9 : kD3Q19;
    const int dims[3] = {sim->nx, sim->ny, sim->nz};
    // (direction, node) the population f_k of node q is read from
    const bool geom = !sim->solid_host.empty();
    // open face a pull enters across (-1: none, or a wall face wins)
    int entry = -1;
    auto source = [&](int k, int x, int y, int z, int& dir) -> size_t {
      const size_t self = size_t(x) + size_t(sim->nx) * (size_t(y) + size_t(sim->ny) * z);
      int c[3] = {x - E[k][0], y - E[k][1], z - E[k][2]};
      entry = -1;
      bool crossed = false, wall = false;
      for (int d = 0; d < 3; ++d) {
        if (c[d] < 0 || c[d] >= dims[d]) {
          if (sim->wall[d]) {
            const int face = 2 * d + (c[d] < 0 ? 0 : 1);
            crossed = true;
            if ((sim->open_mask >> face) & 1) {
              if (entry < 0) entry = face;
            } else {
              wall = true;
            }
            continue;
          }
          c[d] = (c[d] + dims[d]) % dims[d];
        }
      }
      if (crossed) {
        if (wall) entry = -1;
        if (entry >= 0 && geom) {
          // a solid node on the open face continues beyond it: the link whose
          // in-face part comes from a solid node is a wall link
          int t[3] = {x - E[k][0], y - E[k][1], z - E[k][2]};
          t[entry / 2] = entry / 2 == 0 ? x : (entry / 2 == 1 ? y : z);
          bool inside = true;
          for (int d = 0; d < 3; ++d) {
            if (t[d] < 0 || t[d] >= dims[d]) {
              if (sim->wall[d]) inside = false;
              else t[d] = (t[d] + dims[d]) % dims[d];
            }
          }
          const int xyz0[3] = {x, y, z};
          const bool moved = t[0] != xyz0[0] || t[1] != xyz0[1] || t[2] != xyz0[2];
          if (inside && moved &&
              sim->solid_host[size_t(t[0]) + size_t(sim->nx) * (size_t(t[1]) + size_t(sim->ny) * size_t(t[2]))])
            entry = -1;
        }
        dir = (k & 1) ? k + 1 : k - 1;
        return self;
      }
      const size_t src = size_t(c[0]) + size_t(sim->nx) * (size_t(c[1]) + size_t(sim->ny) * c[2]);
      if (geom && sim->solid_host[src]) {   // bounced back from a solid node
        dir = (k & 1) ? k + 1 : k - 1;
        return self;
      }
      dir = k;
      return src;
    };
    if (field == NFLBM_FIELD_G_RAW) std::memset(host_out, 0, size_t(N) * sim->Q * n * sizeof(double));
    // convective outflow: plane N's post-streaming populations are the plane
    // buffers (f [Q-1][P], then g [N-1][Q][P], compute precision)
    std::vector<double> outv;
    int oax = -1, opos = -1;
    if (sim->out_face >= 0) {
      const size_t cnt = (size_t(Qm) + size_t(NE) * sim->Q) * sim->out_plane;
      std::vector<unsigned char> raw(cnt * sim->ts);
      HIPCHK(sim, hipMemcpyAsync(raw.data(), sim->out_buf, raw.size(), hipMemcpyDeviceToHost, sim->stream));
      HIPCHK(sim, hipStreamSynchronize(sim->stream));
      outv.resize(cnt);
      for (size_t i = 0; i < cnt; ++i)
        outv[i] = sim->ts == 8 ? reinterpret_cast<const double*>(raw.data())[i]
                               : static_cast<double>(reinterpret_cast<const float*>(raw.data())[i]);
      oax = sim->out_face / 2;
      opos = (sim->out_face & 1) ? dims[oax] - 1 : 0;
    }
    for (int z = 0; z < sim->nz; ++z)
      for (int y = 0; y < sim->ny; ++y)
        for (int x = 0; x < sim->nx; ++x) {
          const size_t q = size_t(x) + size_t(sim->nx) * (size_t(y) + size_t(sim->ny) * z);
          if (geom && sim->solid_host[q]) {         // no fluid: every population 0
            if (field == NFLBM_FIELD_F_RAW)
              for (int k = 1; k <= Qm; ++k) host_out[size_t(k - 1) * n + q] = 0.0;
            continue;
          }
          const int xyz[3] = {x, y, z};
          if (oax >= 0 && xyz[oax] == opos) {
            const size_t P = sim->out_plane;
            const int t0 = oax == 0 ? 1 : 0, t1 = oax == 2 ? 1 : 2;
            const size_t p = size_t(xyz[t0]) + size_t(dims[t0]) * size_t(xyz[t1]);
            if (field == NFLBM_FIELD_F_RAW) {
              for (int k = 1; k <= Qm; ++k) host_out[size_t(k - 1) * n + q] = outv[size_t(k - 1) * P + p];
            } else {
              for (int i = 0; i < NE; ++i)
                for (int k = 0; k < sim->Q; ++k)
                  host_out[(size_t(sim->uidx[i]) * sim->Q + k) * n + q] =
                      outv[(size_t(Qm) + size_t(i) * sim->Q + k) * P + p];
            }
            continue;
          }
          if (field == NFLBM_FIELD_G_RAW)
            for (int i = 0; i < NE; ++i)
              host_out[size_t(sim->uidx[i]) * sim->Q * n + q] = val(g0buf.data(), q * NE + i, sim->g0s, false);
          for (int k = 1; k <= Qm; ++k) {
            int dir = k;
            const size_t src = source(k, x, y, z, dir);
            if (field == NFLBM_FIELD_F_RAW) {
              double v = val(fbuf.data(), size_t(dir - 1) * fst + src, fbytes, true);
              if (entry >= 0) v += face_fcorr(*sim, entry, k);
              host_out[size_t(k - 1) * n + q] = v;
            } else {
              for (int i = 0; i < NE; ++i) {
                double v = val(gkbuf.data(), size_t(dir - 1) * gst + src * NE + i, sim->fs, true);
                if (entry >= 0) v = face_gsum(*sim, entry, sim->uidx[i], k) - v;
                // moment form before its first step: the initial g_k = 0
                if (entry >= 0 && sim->gform && sim->f_local) v = 0.0;
                host_out[(size_t(sim->uidx[i]) * sim->Q + k) * n + q] = v;
              }
            }
          }
        }
    if (field == NFLBM_FIELD_F_RAW && sim->p_ref != 0.0) {
      const double* W = sim->lat == NFLBM_D2Q9 ? kW2 : kW3;
      for (size_t q = 0; q < n; ++q) {
        if (geom && sim->solid_host[q]) continue;
        for (int k = 1; k <= Qm; ++k) host_out[size_t(k - 1) * n + q] += 3.0 * W[k] * sim->p_ref;
      }
    }
    return NFLBM_OK;
  }
  return fail(sim, NFLBM_EINVAL, "unknown field");
}

// The moment form appends one host-side byte to the checkpoint: whether
// the next step starts from the equilibria set_fields wrote.
size_t state_tail(const nflbm_sim* s) { return s->gform ? 1 : 0; }

int nflbm_state_bytes(nflbm_sim* sim, size_t* bytes) {
  if (!sim || !bytes) return fail(sim, NFLBM_EINVAL, "NULL argument");
  size_t b = 0;
  for (const auto& seg : state_segments(sim)) b += seg.second;
  *bytes = b + state_tail(sim);
  return NFLBM_OK;
}

int nflbm_get_state(nflbm_sim* sim, void* host_raw) {
  if (!sim || !host_raw) return fail(sim, NFLBM_EINVAL, "NULL argument");
  unsigned char* p = static_cast<unsigned char*>(host_raw);
  for (const auto& seg : state_segments(sim)) {
    HIPCHK(sim, hipMemcpyAsync(p, seg.first, seg.second, hipMemcpyDeviceToHost, sim->stream));
    p += seg.second;
  }
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  if (state_tail(sim)) *p = sim->f_local ? 1 : 0;
  return NFLBM_OK;
}

int nflbm_set_state(nflbm_sim* sim, const void* host_raw) {
  if (!sim || !host_raw) return fail(sim, NFLBM_EINVAL, "NULL argument");
  const unsigned char* p = static_cast<const unsigned char*>(host_raw);
  for (const auto& seg : state_segments(sim)) {
    HIPCHK(sim, hipMemcpyAsync(seg.first, p, seg.second, hipMemcpyHostToDevice, sim->stream));
    p += seg.second;
  }
  if (state_tail(sim)) sim->f_local = *p != 0;
  const int rc = refresh_outflow_plane(sim);
  if (rc) return rc;
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  return sim_nan_reset(sim);
}

int nflbm_diagnostics(nflbm_sim* sim, int vcm_component, nflbm_diag* out) {
  if (!sim || !out) return fail(sim, NFLBM_EINVAL, "NULL argument");
  const int rec = reduce_record_len(sim->N);
  if (!sim->red) {
    if (hipMalloc(reinterpret_cast<void**>(&sim->red), size_t(kDiagMaxBlocks + 1) * rec * sizeof(double)) !=
        hipSuccess) {
      sim->red = nullptr;
      return fail(sim, NFLBM_ENOMEM, "cannot allocate the reduction buffer");
    }
  }
  return diag_run(sim, vcm_component, sim->red, kDiagMaxBlocks, sim->red + size_t(kDiagMaxBlocks) * rec, out);
}

int nflbm_set_launch(nflbm_sim* sim, int tx_log2, int zchunk) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  const int l = tx_log2 > 0 ? tx_log2 : sim->tx_log2;
  const int zc = zchunk > 0 ? zchunk : sim->zchunk;
  if (!apply_launch(sim, l, zc)) return fail(sim, NFLBM_EINVAL, "invalid launch shape or LDS too large");
  sim->shape_chosen = true;
  return NFLBM_OK;
}

int nflbm_set_conc_launch(nflbm_sim* sim, int tx_log2, int zchunk) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  const int l = tx_log2 > 0 ? tx_log2 : sim->ctx_log2;
  const int zc = zchunk > 0 ? zchunk : sim->czchunk;
  if (!apply_conc_launch(sim, l, zc)) return fail(sim, NFLBM_EINVAL, "invalid launch shape or LDS too large");
  sim->shape_chosen = true;
  return NFLBM_OK;
}

int nflbm_get_conc_launch(nflbm_sim* sim, int* tx_log2, int* zchunk) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  if (tx_log2) *tx_log2 = sim->ctx_log2;
  if (zchunk) *zchunk = sim->czchunk;
  return NFLBM_OK;
}

int nflbm_get_launch(nflbm_sim* sim, int* tx_log2, int* zchunk, int* lds_limit) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  if (tx_log2) *tx_log2 = sim->tx_log2;
  if (zchunk) *zchunk = sim->zchunk;
  if (lds_limit) *lds_limit = static_cast<int>(sim->lds_max);
  return NFLBM_OK;
}

int nflbm_storage_form(const nflbm_sim* sim) { return sim ? sim->gform : NFLBM_EINVAL; }

int nflbm_f_storage_form(const nflbm_sim* sim) { return sim ? sim->fform : NFLBM_EINVAL; }

int nflbm_bytes_per_node(nflbm_sim* sim, double* bytes) {
  if (!sim || !bytes) return fail(sim, NFLBM_EINVAL, "NULL argument");
  const double Qm = sim->Q - 1, NE = sim->NE;
  double b;
  const double ts = double(sim->ts), rs = double(sim->rs);
  if (sim->fform) {
    // record form of f: the reconstruction reads C, mu~, (v, -3/2 v.v) and
    // (fB, F) and writes C, E_B and the four f moments; the update reads C,
    // E_B and the f moments and writes mu~, (v, -3/2 v.v) and (fB, F)
    b = (NE * ts + (NE + 4 + 4) * rs) + ((NE + 1) * ts + 4 * rs) + ((NE + 1) * ts + 4 * rs) +
        (NE + 4 + 4) * rs;
  } else if (sim->gform) {
    // f read and written; reconstruction reads C, mu~, (v, -3/2 v.v) and
    // writes C, E_B; the update reads C, E_B and writes mu~, (v, -3/2 v.v)
    b = 2.0 * Qm * sim->fs + (NE * ts + (NE + 4) * rs) + 2.0 * (NE + 1) * ts + (NE + 4) * rs;
  } else {
    b = 2.0 * (Qm * sim->fs + NE * sim->g0s + NE * Qm * sim->fs) + 2.0 * (NE + 1) * sim->ts;
    if (sim->step_flags & kFlagNeedG) b += NE * Qm * sim->fs;
    // concentration-dependent mobility: potentials read C and write N values;
    // the source reads them and C, rewrites the moving populations and g0
    if (sim->c2c2) b += (NE + sim->N) * sim->ts + (sim->N + NE) * sim->ts + 2.0 * NE * Qm * sim->fs + NE * sim->g0s;
  }
  if (sim->step_flags & kFlagNoHydro) b -= 2.0 * Qm * sim->fs;   // f neither read nor written
  *bytes = b;
  return NFLBM_OK;
}


int nflbm_autotune(nflbm_sim* sim, const char* cache_path) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  const std::string key = sim_key(sim);
  std::vector<int> best = {sim->tx_log2, sim->zchunk, sim->ctx_log2, sim->czchunk};
  if (cache_lookup(cache_path, key, &best)) {
    if (apply_launch(sim, best[0], best[1]) && apply_conc_launch(sim, best[2], best[3])) {
      sim->shape_chosen = true;
      return NFLBM_OK;
    }
  }
  std::vector<std::pair<int, int>> cands;
  for (int l : {4, 6}) {
    if (sim->lat == NFLBM_D3Q19) {
      for (int zc = 1; zc <= sim->nz; zc *= 2) cands.emplace_back(l, zc);
      if ((sim->nz & (sim->nz - 1)) != 0) cands.emplace_back(l, sim->nz);
    } else {
      cands.emplace_back(l, 1);
    }
  }
  SavedState st;
  int rc = save_state(sim, &st);
  if (rc != NFLBM_OK) {
    (void)restore_state(sim, &st);
    return rc;
  }
  double bpn = 0.0;
  (void)nflbm_bytes_per_node(sim, &bpn);
  const long long K = tune_steps(double(sim->n), bpn);
  const int keep[4] = {sim->tx_log2, sim->zchunk, sim->ctx_log2, sim->czchunk};
  best = {keep[0], keep[1], keep[2], keep[3]};
  // the update's shape by the update's own time, then the reconstruction's
  // by the rest of the step, the other kernel's shape held fixed
  for (int pass = 0; pass < 2 && rc == NFLBM_OK; ++pass) {
    double best_ms = 1e300;
    for (const auto& c : cands) {
      const bool ok = pass == 0 ? apply_launch(sim, c.first, c.second) : apply_conc_launch(sim, c.first, c.second);
      if (!ok) continue;
      rc = nflbm_step(sim, 2);
      double ms = 0.0, mu = 0.0;
      if (rc == NFLBM_OK) rc = nflbm_step_timed(sim, K, &ms, &mu);
      if (rc != NFLBM_OK) break;
      const double t = pass == 0 ? mu : ms - mu;
      if (t < best_ms) {
        best_ms = t;
        best[2 * pass] = c.first;
        best[2 * pass + 1] = c.second;
      }
    }
    if (pass == 0 && !apply_launch(sim, best[0], best[1])) (void)apply_launch(sim, keep[0], keep[1]);
  }
  const int rc2 = restore_state(sim, &st);
  if (!apply_launch(sim, best[0], best[1])) (void)apply_launch(sim, keep[0], keep[1]);
  if (!apply_conc_launch(sim, best[2], best[3])) (void)apply_conc_launch(sim, keep[2], keep[3]);
  if (rc != NFLBM_OK) return rc;
  if (rc2 != NFLBM_OK) return rc2;
  sim->shape_chosen = true;
  cache_store(cache_path, key, best);
  return NFLBM_OK;
}

int nflbm_batch_create(const nflbm_config* cfgs, int count, nflbm_batch** out) {
  if (!cfgs || !out || count < 1) return bfail(nullptr, NFLBM_EINVAL, "batch needs count >= 1 configurations");
  *out = nullptr;
  for (int i = 1; i < count; ++i)
    if (cfgs[i].lattice != cfgs[0].lattice || cfgs[i].ncomp != cfgs[0].ncomp ||
        cfgs[i].precision != cfgs[0].precision)
      return bfail(nullptr, NFLBM_EINVAL, "batch members must share lattice, ncomp and precision");
  // one storage form of g for every member: populations if any member needs
  // them (some tau_g != 1, the concentration-dependent mobility, or asked for)
  std::vector<nflbm_config> cc(cfgs, cfgs + count);
  bool pop = false;
  for (const auto& c : cc) {
    if (c.flags & (NFLBM_FLAG_G_POPULATIONS | NFLBM_FLAG_C2C2_MOBILITY)) pop = true;
    for (int i = 0; c.tau_g && i < c.ncomp; ++i)
      if (c.tau_g[i] != 1.0) pop = true;
  }
  if (pop)
    for (auto& c : cc) c.flags |= NFLBM_FLAG_G_POPULATIONS;
  nflbm_batch* b = new nflbm_batch();
  b->lat = cfgs[0].lattice;
  b->N = cfgs[0].ncomp;
  b->store = cfgs[0].precision;
  auto cleanup = [&](int code, const std::string& msg) {
    for (nflbm_sim* m : b->members) nflbm_destroy(m);
    if (b->params) (void)hipFree(b->params);
    if (b->nanflag) (void)hipFree(b->nanflag);
    if (b->nan_host) (void)hipHostFree(b->nan_host);
    if (b->nan_ev) (void)hipEventDestroy(b->nan_ev);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    delete b;
    return bfail(nullptr, code, msg);
  };
  for (int attempt = 0; attempt < 2; ++attempt) {
    for (int i = 0; i < count; ++i) {
      nflbm_sim* m = nullptr;
      const int rc = nflbm_create(&cc[i], &m);
      if (rc != NFLBM_OK) return cleanup(rc, "member " + std::to_string(i) + ": " + nflbm_last_error(nullptr));
      m->in_batch = true;
      b->members.push_back(m);
    }
    bool same = true;
    for (nflbm_sim* m : b->members) same = same && m->gform == b->members[0]->gform;
    if (same) break;
    // a member fell back to populations (its LDS window): all do
    for (nflbm_sim* m : b->members) nflbm_destroy(m);
    b->members.clear();
    for (auto& c : cc) c.flags |= NFLBM_FLAG_G_POPULATIONS;
  }
  for (nflbm_sim* m : b->members) {
    b->nodes += static_cast<long long>(m->n);
    if (m->wall[0] || m->wall[1] || m->wall[2]) b->walls = 1;
  }
  if (hipStreamCreate(&b->own_stream) != hipSuccess) {
    b->own_stream = nullptr;
    return cleanup(NFLBM_EDEVICE, "cannot create the batch stream");
  }
  b->stream = b->own_stream;
  for (nflbm_sim* m : b->members) m->stream = b->stream;
  // coefficient tables of all members in one array
  const size_t psize = b->members[0]->ts == 8 ? sizeof(DevParams<double>) : sizeof(DevParams<float>);
  if (hipMalloc(&b->params, psize * count) != hipSuccess) {
    b->params = nullptr;
    return cleanup(NFLBM_ENOMEM, "cannot allocate the batch coefficient tables");
  }
  for (int i = 0; i < count; ++i)
    if (hipMemcpy(static_cast<char*>(b->params) + psize * i, b->members[i]->params, psize,
                  hipMemcpyDeviceToDevice) != hipSuccess)
      return cleanup(NFLBM_EDEVICE, "cannot copy the coefficient tables");
  if (hipMalloc(reinterpret_cast<void**>(&b->nanflag), sizeof(int)) != hipSuccess ||
      hipMemset(b->nanflag, 0, sizeof(int)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->nan_host), sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&b->nan_ev, hipEventDisableTiming) != hipSuccess)
    return cleanup(NFLBM_ENOMEM, "cannot allocate the batch NaN flag");
  *b->nan_host = 0;
  // default tile: 64 x 4 unless some member is at most 16 wide or the window
  // does not fit
  int l = 6;
  for (nflbm_sim* m : b->members)
    if (m->nx <= 16) l = 4;
  if (!batch_tile_fits(b, l)) l = 4;
  b->tx_log2 = l;
  const int rc = build_batch_tables(b, true);
  if (rc != NFLBM_OK) {
    const std::string msg = b->err;
    free_batch_tables(b);
    return cleanup(rc, msg);
  }
  *out = b;
  return NFLBM_OK;
}

void nflbm_batch_destroy(nflbm_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  destroy_graphs(b);
  free_batch_tables(b);
  if (b->params) (void)hipFree(b->params);
  if (b->nanflag) (void)hipFree(b->nanflag);
  if (b->nan_host) (void)hipHostFree(b->nan_host);
  if (b->nan_ev) (void)hipEventDestroy(b->nan_ev);
  for (nflbm_sim* m : b->members) {
    m->stream = nullptr;
    nflbm_destroy(m);
  }
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  delete b;
}

int nflbm_batch_count(const nflbm_batch* b) { return b ? static_cast<int>(b->members.size()) : 0; }

nflbm_sim* nflbm_batch_member(nflbm_batch* b, int idx) {
  if (!b || idx < 0 || idx >= static_cast<int>(b->members.size())) {
    bfail(b, NFLBM_EINVAL, "member index out of range");
    return nullptr;
  }
  return b->members[idx];
}

int nflbm_batch_set_stream(nflbm_batch* b, void* stream) {
  if (!b) return bfail(nullptr, NFLBM_EINVAL, "NULL batch");
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  b->stream = stream ? static_cast<hipStream_t>(stream) : b->own_stream;
  for (nflbm_sim* m : b->members) m->stream = b->stream;
  return NFLBM_OK;
}

int nflbm_batch_set_fields(nflbm_batch* b, int idx, const double* C, const double* v, const double* P) {
  nflbm_sim* m = nflbm_batch_member(b, idx);
  if (!m) return NFLBM_EINVAL;
  const int rc = nflbm_set_fields(m, C, v, P);
  return rc == NFLBM_OK ? batch_nan_reset(b) : bfail(b, rc, m->err);
}

int nflbm_batch_get_field(nflbm_batch* b, int idx, int field, double* host_out) {
  nflbm_sim* m = nflbm_batch_member(b, idx);
  if (!m) return NFLBM_EINVAL;
  const int rc = nflbm_get_field(m, field, host_out);
  return rc == NFLBM_OK ? rc : bfail(b, rc, m->err);
}

int nflbm_batch_step(nflbm_batch* b, long long nsteps, int mode) {
  if (!b) return bfail(nullptr, NFLBM_EINVAL, "NULL batch");
  if (nsteps < 0) return bfail(b, NFLBM_EINVAL, "nsteps < 0");
  if (mode != NFLBM_BATCH_LAUNCH && mode != NFLBM_BATCH_GRAPH && mode != NFLBM_BATCH_PER_SIM)
    return bfail(b, NFLBM_EINVAL, "unknown batch mode");
  return batch_run(b, nsteps, mode);
}

int nflbm_batch_step_timed(nflbm_batch* b, long long nsteps, int mode, double* ms) {
  if (!b || !ms) return bfail(b, NFLBM_EINVAL, "NULL argument");
  if (nsteps < 0) return bfail(b, NFLBM_EINVAL, "nsteps < 0");
  if (mode != NFLBM_BATCH_LAUNCH && mode != NFLBM_BATCH_GRAPH && mode != NFLBM_BATCH_PER_SIM)
    return bfail(b, NFLBM_EINVAL, "unknown batch mode");
  hipEvent_t e0, e1;
  BHIPCHK(b, hipEventCreate(&e0));
  BHIPCHK(b, hipEventCreate(&e1));
  BHIPCHK(b, hipEventRecord(e0, b->stream));
  int rc = batch_run(b, nsteps, mode);
  if (rc == NFLBM_OK) {
    BHIPCHK(b, hipEventRecord(e1, b->stream));
    BHIPCHK(b, hipEventSynchronize(e1));
    float t = 0.f;
    BHIPCHK(b, hipEventElapsedTime(&t, e0, e1));
    *ms = t;
    BHIPCHK(b, nan_poll(&b->nan_pending, &b->nan_seen, b->nan_host, b->nan_ev, true));
    if (b->nan_seen) rc = bfail(b, NFLBM_ENUMERIC, "a NaN or Inf appeared in a member's state");
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int nflbm_batch_set_launch(nflbm_batch* b, int tx_log2, int graph_steps) {
  if (!b) return bfail(nullptr, NFLBM_EINVAL, "NULL batch");
  const int l = tx_log2 > 0 ? tx_log2 : b->tx_log2;
  const int g = graph_steps > 0 ? graph_steps : b->graph_steps;
  if (l != 4 && l != 6) return bfail(b, NFLBM_EINVAL, "tx_log2 must be 4 or 6");
  if (g < 2 || (g & 1)) return bfail(b, NFLBM_EINVAL, "graph_steps must be even and >= 2");
  if (!batch_tile_fits(b, l)) return bfail(b, NFLBM_EINVAL, "LDS window too large for this tile");
  const bool shape = l != b->tx_log2 || g != b->graph_steps;
  b->tx_log2 = l;
  b->graph_steps = g;
  return shape ? build_batch_tables(b, true) : NFLBM_OK;
}

int nflbm_batch_get_launch(nflbm_batch* b, int* tx_log2, int* graph_steps, int* blocks_update) {
  if (!b) return bfail(nullptr, NFLBM_EINVAL, "NULL batch");
  if (tx_log2) *tx_log2 = b->tx_log2;
  if (graph_steps) *graph_steps = b->graph_steps;
  if (blocks_update) *blocks_update = b->blocks_update;
  return NFLBM_OK;
}

int nflbm_batch_nodes(const nflbm_batch* b, long long* nodes) {
  if (!b || !nodes) return bfail(nullptr, NFLBM_EINVAL, "NULL argument");
  *nodes = b->nodes;
  return NFLBM_OK;
}

int nflbm_batch_autotune(nflbm_batch* b, const char* cache_path) {
  if (!b) return bfail(nullptr, NFLBM_EINVAL, "NULL batch");
  std::ostringstream ko;
  unsigned long long h = 1469598103934665603ULL;  // FNV-1a over the member shapes
  for (nflbm_sim* m : b->members)
    for (int v : {m->nx, m->ny, m->nz, m->wall[0], m->wall[1], m->wall[2], m->step_flags}) {
      h ^= static_cast<unsigned long long>(static_cast<unsigned>(v));
      h *= 1099511628211ULL;
    }
  ko << "batch lat=" << b->lat << " N=" << b->N << " store=" << b->store << " count=" << b->members.size()
     << " nodes=" << b->nodes << " shapes=" << std::hex << h << std::dec << " dev=" << device_tag();
  const std::string key = ko.str();
  std::vector<int> best = {b->tx_log2};
  if (cache_lookup(cache_path, key, &best)) return nflbm_batch_set_launch(b, best[0], 0);
  std::vector<SavedState> saved(b->members.size());
  int rc = NFLBM_OK;
  for (size_t i = 0; i < b->members.size() && rc == NFLBM_OK; ++i) {
    rc = save_state(b->members[i], &saved[i]);
    if (rc != NFLBM_OK) rc = bfail(b, rc, b->members[i]->err);
  }
  double bpn = 0.0;
  (void)nflbm_bytes_per_node(b->members[0], &bpn);
  const long long K = std::max<long long>(tune_steps(double(b->nodes), bpn), b->graph_steps);
  double best_ms = 1e300;
  best = {b->tx_log2};
  for (int l : {4, 6}) {
    if (rc != NFLBM_OK) break;
    if (!batch_tile_fits(b, l)) continue;
    rc = nflbm_batch_set_launch(b, l, 0);
    double ms = 0.0;
    if (rc == NFLBM_OK) rc = batch_run(b, b->graph_steps, NFLBM_BATCH_GRAPH);  // warm-up and capture
    if (rc == NFLBM_OK) rc = nflbm_batch_step_timed(b, K, NFLBM_BATCH_GRAPH, &ms);
    if (rc == NFLBM_OK && ms < best_ms) {
      best_ms = ms;
      best = {l};
    }
  }
  for (size_t i = 0; i < b->members.size(); ++i) {
    const int r2 = restore_state(b->members[i], &saved[i]);
    if (r2 != NFLBM_OK && rc == NFLBM_OK) rc = bfail(b, r2, b->members[i]->err);
  }
  if (rc != NFLBM_OK) return rc;
  rc = nflbm_batch_set_launch(b, best[0], 0);
  if (rc != NFLBM_OK) return rc;
  rc = build_batch_tables(b, false);
  if (rc != NFLBM_OK) return rc;
  cache_store(cache_path, key, best);
  return NFLBM_OK;
}

const char* nflbm_batch_last_error(const nflbm_batch* b) { return b ? b->err.c_str() : g_thread_error.c_str(); }


int nflbm_device_bytes(const nflbm_config* cfg, size_t* bytes) {
  if (!cfg || !bytes) return fail(nullptr, NFLBM_EINVAL, "NULL argument");
  nflbm_sim s;
  const int rc = plan_sim(cfg, &s);
  if (rc != NFLBM_OK) return rc;
  size_t total = 0;
  for (const auto& a : state_arrays(&s)) total += align_up(a.second);
  *bytes = total;
  return NFLBM_OK;
}

int nflbm_bind_state(nflbm_sim* sim, void* dev_ptr, size_t bytes) {
  if (!sim || !dev_ptr) return fail(sim, NFLBM_EINVAL, "NULL argument");
  if (sim->in_batch) return fail(sim, NFLBM_EINVAL, "batch members keep library memory");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kBindAlign != 0)
    return fail(sim, NFLBM_EINVAL, "dev_ptr must be 256-byte aligned");
  auto arrays = state_arrays(sim);
  size_t total = 0;
  for (const auto& a : arrays) total += align_up(a.second);
  if (bytes < total) return fail(sim, NFLBM_EINVAL, "buffer smaller than nflbm_device_bytes");
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  unsigned char* base = static_cast<unsigned char*>(dev_ptr);
  if (base == static_cast<unsigned char*>(*arrays[0].first)) return NFLBM_OK;   // already bound here
  size_t off = 0;
  std::vector<void*> old;
  for (auto& a : arrays) {
    void* dst = base + off;
    HIPCHK(sim, hipMemcpyAsync(dst, *a.first, a.second, hipMemcpyDeviceToDevice, sim->stream));
    old.push_back(*a.first);
    *a.first = dst;
    off += align_up(a.second);
  }
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  if (!sim->borrowed)
    for (void* p : old) (void)hipFree(p);
  sim->borrowed = true;
  return NFLBM_OK;
}

int nflbm_get_coeffs(const nflbm_sim* sim, double* alpha, double* gamma) {
  if (!sim) return fail(nullptr, NFLBM_EINVAL, "NULL sim");
  const int N = sim->N;
  for (int i = 0; i < N; ++i) {
    if (gamma) gamma[i] = sim->co.gamma[i];
    for (int j = 0; j < N; ++j)
      if (alpha) alpha[i * N + j] = sim->co.alpha[i][j];
  }
  return NFLBM_OK;
}


int nflbm_domain_size(nflbm_sim* sim, double* L) {
  if (!sim || !L) return fail(sim, NFLBM_EINVAL, "NULL argument");
  int rc = compute_fields(sim);
  if (rc) return rc;
  const int N = sim->N;
  const long long n = static_cast<long long>(sim->n);
  const long long nc = static_cast<long long>(sim->nz) * sim->ny * (sim->nx / 2 + 1);
  const int blocks = 256;
  if (!sim->fft_made) {
    bool ok = hipMalloc(reinterpret_cast<void**>(&sim->lam), size_t(N) * n * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&sim->spec, size_t(N) * nc * 2 * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&sim->spart), size_t(N) * blocks * 2 * sizeof(double)) == hipSuccess;
    if (!ok) return fail(sim, NFLBM_ENOMEM, "cannot allocate the domain-size buffers");
    int dims3[3] = {sim->nz, sim->ny, sim->nx};
    int dims2[2] = {sim->ny, sim->nx};
    const bool three = sim->nz > 1;
    hipfftResult r = hipfftPlanMany(&sim->fft, three ? 3 : 2, three ? dims3 : dims2, nullptr, 1, static_cast<int>(n),
                                    nullptr, 1, static_cast<int>(nc), HIPFFT_D2Z, N);
    if (r != HIPFFT_SUCCESS) return fail(sim, NFLBM_EDEVICE, "hipfftPlanMany failed");
    sim->fft_made = true;
  }
  if (hipfftSetStream(sim->fft, sim->stream) != HIPFFT_SUCCESS) return fail(sim, NFLBM_EDEVICE, "hipfftSetStream failed");
  HIPCHK(sim, launch_lambda(sim->fields, sim->lam, static_cast<long long>(N) * n, sim->stream));
  if (hipfftExecD2Z(sim->fft, sim->lam, static_cast<hipfftDoubleComplex*>(sim->spec)) != HIPFFT_SUCCESS)
    return fail(sim, NFLBM_EDEVICE, "hipfftExecD2Z failed");
  HIPCHK(sim, launch_spectrum(sim->spec, N, sim->nx, sim->ny, sim->nz, nc, blocks, sim->spart, sim->stream));
  std::vector<double> part(size_t(N) * blocks * 2);
  HIPCHK(sim, hipMemcpyAsync(part.data(), sim->spart, part.size() * sizeof(double), hipMemcpyDeviceToHost, sim->stream));
  HIPCHK(sim, hipStreamSynchronize(sim->stream));
  const double two_pi = 6.283185307179586;
  for (int i = 0; i < N; ++i) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < blocks; ++k) {
      a += part[(size_t(i) * blocks + k) * 2];
      b += part[(size_t(i) * blocks + k) * 2 + 1];
    }
    L[i] = b > 0.0 ? two_pi * a / b : 0.0;
  }
  return NFLBM_OK;
}

}  // extern "C"
