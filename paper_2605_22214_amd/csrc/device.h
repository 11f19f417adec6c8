// Device-side building blocks shared by the kernel sources: the lattices,
// the storage types of each precision, vector and nontemporal node
// accesses, the free-energy polynomials, the equilibrium pair terms and the
// pull-streaming neighbour rules.  Included by device code only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace nflbm {

// ---------------------------------------------------------------- lattices
struct D2Q9 {
  static constexpr int Q = 9, DIM = 2;
  static constexpr int e[9][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                  {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

struct D3Q19 {
  static constexpr int Q = 19, DIM = 3;
  static constexpr int e[19][3] = {
      {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
      {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
      {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};
// In both sets the opposite of direction k (k >= 1) is k + 1 for odd k.
__host__ __device__ constexpr int opposite(int k) { return (k & 1) ? k + 1 : k - 1; }
// Index of the direction (ex, ey, ez) in set L, or -1.
template <class L>
__host__ __device__ constexpr int direction_of(int ex, int ey, int ez) {
  for (int k = 0; k < L::Q; ++k)
    if (L::e[k][0] == ex && L::e[k][1] == ey && L::e[k][2] == ez) return k;
  return -1;
}

// ----------------------------------------------------------- storage types
template <int ST> struct StoreT;
// ld / pack / unpack convert between a stored moving population and its
// value; ld_raw / pack_raw move the stored number itself, which is the value
// times `scale` (a power of two, so arithmetic on raw numbers scaled by it
// rounds exactly as on the values).
// RS is the type of the moment form's node records (mu~, (v, -3/2 v.v),
// (fB, F), the f moments; C and E_B keep the compute type), stored as the
// value times mu_scale (mu~) or vel_scale (the others).
template <> struct StoreT<kStoreF64> {
  using T = double; using FS = double; using G0S = double; using RS = double;
  static constexpr double scale = 1.0, mu_scale = 1.0, vel_scale = 1.0;
  static __device__ __forceinline__ T ld(const FS* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ FS pack(T v) { return v; }
  static __device__ __forceinline__ T unpack(FS v) { return v; }
  static __device__ __forceinline__ T ld_raw(const FS* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ FS pack_raw(T v) { return v; }
};
template <> struct StoreT<kStoreF32> {
  using T = float; using FS = float; using G0S = float; using RS = float;
  static constexpr float scale = 1.0f, mu_scale = 1.0f, vel_scale = 1.0f;
  static __device__ __forceinline__ T ld(const FS* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ FS pack(T v) { return v; }
  static __device__ __forceinline__ T unpack(FS v) { return v; }
  static __device__ __forceinline__ T ld_raw(const FS* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ FS pack_raw(T v) { return v; }
};
template <> struct StoreT<kStoreF16S> {
  using T = float; using FS = _Float16; using G0S = float; using RS = _Float16;
  static constexpr float scale = kHalfScale, mu_scale = kRecMuScale, vel_scale = kRecVelScale;
  static __device__ __forceinline__ T ld(const FS* p, size_t i) {
    return static_cast<float>(p[i]) * (1.0f / kHalfScale);
  }
  static __device__ __forceinline__ FS pack(T v) { return static_cast<_Float16>(v * kHalfScale); }
  static __device__ __forceinline__ T unpack(FS v) { return static_cast<float>(v) * (1.0f / kHalfScale); }
  static __device__ __forceinline__ T ld_raw(const FS* p, size_t i) { return static_cast<float>(p[i]); }
  static __device__ __forceinline__ FS pack_raw(T v) { return static_cast<_Float16>(v); }
};

// ------------------------------------------------- per-node vector access
// The NE values a node holds for one direction are contiguous; groups of 4,
// 8, 16 or 32 bytes move with single vector instructions.  Node offsets are
// multiples of the group size, so these accesses are aligned.
template <class E, int NE>
__device__ __forceinline__ void vld(const E* p, E (&o)[NE]) {
  constexpr int B = int(sizeof(E)) * NE;
  if constexpr (B == 4) {
    const uint32_t t = *reinterpret_cast<const uint32_t*>(p);
    __builtin_memcpy(o, &t, 4);
  } else if constexpr (B == 8) {
    const uint2 t = *reinterpret_cast<const uint2*>(p);
    __builtin_memcpy(o, &t, 8);
  } else if constexpr (B == 16) {
    const uint4 t = *reinterpret_cast<const uint4*>(p);
    __builtin_memcpy(o, &t, 16);
  } else if constexpr (B == 32) {
    uint4 t[2];
    t[0] = reinterpret_cast<const uint4*>(p)[0];
    t[1] = reinterpret_cast<const uint4*>(p)[1];
    __builtin_memcpy(o, t, 32);
  } else {
#pragma unroll
    for (int e = 0; e < NE; ++e) o[e] = p[e];
  }
}

template <class E, int NE>
__device__ __forceinline__ void vst(E* p, const E (&v)[NE]) {
  constexpr int B = int(sizeof(E)) * NE;
  if constexpr (B == 4) {
    uint32_t t;
    __builtin_memcpy(&t, v, 4);
    *reinterpret_cast<uint32_t*>(p) = t;
  } else if constexpr (B == 8) {
    uint2 t;
    __builtin_memcpy(&t, v, 8);
    *reinterpret_cast<uint2*>(p) = t;
  } else if constexpr (B == 16) {
    uint4 t;
    __builtin_memcpy(&t, v, 16);
    *reinterpret_cast<uint4*>(p) = t;
  } else if constexpr (B == 32) {
    uint4 t[2];
    __builtin_memcpy(t, v, 32);
    reinterpret_cast<uint4*>(p)[0] = t[0];
    reinterpret_cast<uint4*>(p)[1] = t[1];
  } else {
#pragma unroll
    for (int e = 0; e < NE; ++e) p[e] = v[e];
  }
}

// Nontemporal forms for streams touched once per step: the populations the
// reconstruction gathers and the post-collision populations the update
// writes (re-read only by the next step's reconstruction).  Streaming stores
// also leave L2 free of dirty lines for the reconstruction that follows.
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));

template <class E, int NE>
__device__ __forceinline__ void vld_nt(const E* p, E (&o)[NE]) {
  constexpr int B = int(sizeof(E)) * NE;
  if constexpr (B == 4) {
    const unsigned t = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
    __builtin_memcpy(o, &t, 4);
  } else if constexpr (B == 8) {
    const nt_u2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(p));
    __builtin_memcpy(o, &t, 8);
  } else if constexpr (B == 16) {
    const nt_u4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p));
    __builtin_memcpy(o, &t, 16);
  } else {
    // wider records move as two 16-byte halves from different instructions;
    // a streaming hint would drop the line between them (measured: FP64
    // reconstruction 10% slower), so they take the cached path
    vld<E, NE>(p, o);
  }
}

template <class E, int NE>
__device__ __forceinline__ void vst_nt(E* p, const E (&v)[NE]) {
  constexpr int B = int(sizeof(E)) * NE;
  if constexpr (B == 4) {
    unsigned t;
    __builtin_memcpy(&t, v, 4);
    __builtin_nontemporal_store(t, reinterpret_cast<unsigned*>(p));
  } else if constexpr (B == 8) {
    nt_u2 t;
    __builtin_memcpy(&t, v, 8);
    __builtin_nontemporal_store(t, reinterpret_cast<nt_u2*>(p));
  } else if constexpr (B == 16) {
    nt_u4 t;
    __builtin_memcpy(&t, v, 16);
    __builtin_nontemporal_store(t, reinterpret_cast<nt_u4*>(p));
  } else {
    vst<E, NE>(p, v);   // as in vld_nt
  }
}

// A uniform value the compiler must treat as new at this point: direction
// offsets derived from it are formed where they are used instead of being
// hoisted out of the z loop, where dozens of 64-bit bases would stay live in
// scalar registers and spill.
__device__ __forceinline__ size_t fresh(size_t v) {
  asm volatile("" : "+s"(v));
  return v;
}
// Read-only tables seen through the constant address space: uniform reads
// become scalar loads with immediate offsets, and the pointer is fresh at the
// point of use (see above).
#if defined(__HIP_DEVICE_COMPILE__)
#define NFLBM_CONST __attribute__((address_space(4)))
#else
#define NFLBM_CONST
#endif
template <class E>
__device__ __forceinline__ const NFLBM_CONST E* fresh_const(const E* p) {
  const NFLBM_CONST E* c = (const NFLBM_CONST E*)(const NFLBM_GLOBAL E*)p;
  asm volatile("" : "+s"(c));
  return c;
}

template <class E>
__device__ __forceinline__ void st_nt(E* p, E v) {
  __builtin_nontemporal_store(v, p);
}

template <class T>
__device__ __forceinline__ T fpoly(T c) {
  const T d = T(1) - c;
  return c * c * d * d;
}
template <class T>
__device__ __forceinline__ T fprime(T c) {
  return (T(2) * c) * fma(T(2) * c, c, fma(-T(3), c, T(1)));
}

// E_B = sum_{i<j} beta_ij [f(C_i) + f(C_j) - f(C_i + C_j)]  (Eq. FreeEnergy),
// with f(c) = c^2 (1 - c)^2 expanded per pair: for a = C_i, b = C_j, s = a + b,
//   f(a) + f(b) - f(a + b) = a b [2 a b - 2 + s (6 - 4 s)],
// seven operations a pair instead of three quartics, and no cancellation
// between them (the pair term vanishes exactly with a or b).
template <int NC, class T, class PT>
__device__ __forceinline__ T bulk_energy(const T (&c)[NC], const PT& P) {
  T e = T(0);
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = i + 1; j < NC; ++j) {
      const T s = c[i] + c[j];
      const T ab = c[i] * c[j];
      const T g2 = fma(s, fma(-T(4), s, T(6)), fma(T(2), ab, -T(2)));
      e = fma(P.beta[i][j] * ab, g2, e);
    }
  return e;
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ------------------------------------------------- equilibrium pair terms
// e_k . a for a 3-vector a, summed over the nonzero components of e_k from
// the first one on.
template <class L, class T>
__device__ __forceinline__ T proj(int k, const T (&a)[3]) {
  T r = T(0);
  bool first = true;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (L::e[k][d] != 0) {
      const T t = (L::e[k][d] > 0) ? a[d] : -a[d];
      r = first ? t : r + t;
      first = false;
    }
  return r;
}

// s_k(v) = w_k [3 e_k.v + 4.5 (e_k.v)^2 - 1.5 v.v] (Eqs. feq, geq) for
// direction kd, formed through the odd member k of its pair {k, k+1} so that
// both members come from the same ev = e_k.v and quad; base_s = -1.5 v.v.
// Every kernel that forms s_k goes through here, so the reconstruction of the
// moment form forms each s_k exactly as the update does.
template <class L, class T>
__device__ __forceinline__ T quad_term(T ev, T base_s) {
  return fma(T(4.5) * ev, ev, base_s);
}
template <class L, class T>
__device__ __forceinline__ T s_pair_member(int kd, T ev, T quad) {
  return static_cast<T>(L::w[kd]) * fma((kd & 1) ? T(3) : -T(3), ev, quad);
}

// Post-collision population of an evolved component for tau_g = 1, i.e. its
// equilibrium C s_k - w_k m mu~ (Eq. geq, rest-population reading), as the
// update forms it.  The moment form keeps it in the compute precision; with
// FP16S (binary16 moving populations) it thereby skips that rounding, since
// it stores no populations of g.
template <class T>
__device__ __forceinline__ T g_post(T c, T s, T mmu) {
  return fma(c, s, -mmu);
}
// Post-collision rest population for tau_g = 1: g^eq_0 = C_i (1 + s_0) +
// (1 - w_0) m mu~_i (Eq. geq, rest-population reading), with m0mu =
// (1 - w_0) m mu~_i.  The moment form uses it directly; the population form
// stores C_i minus its stored moving populations instead, which equals it in
// exact arithmetic and keeps node mass to one rounding of binary16 storage.
template <class T>
__device__ __forceinline__ T g_rest(T c, T s0, T m0mu) {
  return fma(c, s0, c) + m0mu;
}
// 1 - w_0 as the sum of the moving weights in precision T, in direction
// order.  The moving populations carry -w_k m mu~ with w_k rounded to T; the
// rest population must carry exactly their sum, or every step would shift the
// mass of a component by m mu~ times the rounding of the weights (3e-8 per
// step in float, measured as a drift against FP64).
template <class L, class T>
__host__ __device__ constexpr T moving_weight_sum() {
  T s = T(0);
  for (int k = 1; k < L::Q; ++k) s += static_cast<T>(L::w[k]);
  return s;
}

// ------------------------------------------------------- streaming sources
// Offsets of the neighbour rows of a node: x-1, x, x+1 with periodic wrap
// (y and z pre-multiplied by the row and plane strides), and which faces of
// the node are walls.
struct Nbr {
  uint32_t xo[3], yo[3], zo[3];
  bool wlo[3], whi[3];
  bool geom;      // solid geometry given: pm decides, the faces are folded in
  uint32_t pm;    // its pull mask (StepArgs::bb) of this node
};

template <class L, bool WALLS>
__device__ __forceinline__ Nbr neighbours(int x, int y, int z, const StepArgs& a) {
  constexpr bool D3 = (L::DIM == 3);
  Nbr b;
  const uint32_t nx = a.nx, nxy = uint32_t(a.nx) * uint32_t(a.ny);
  b.xo[0] = x - 1; b.xo[1] = x; b.xo[2] = x + 1;
  b.yo[0] = y - 1; b.yo[1] = y; b.yo[2] = y + 1;
  b.zo[0] = z - 1; b.zo[1] = z; b.zo[2] = z + 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) b.wlo[d] = b.whi[d] = false;
  if (x == 0) { if (WALLS && a.wall_x) b.wlo[0] = true; else b.xo[0] = a.nx - 1; }
  if (x == a.nx - 1) { if (WALLS && a.wall_x) b.whi[0] = true; else b.xo[2] = 0; }
  if (y == 0) { if (WALLS && a.wall_y) b.wlo[1] = true; else b.yo[0] = a.ny - 1; }
  if (y == a.ny - 1) { if (WALLS && a.wall_y) b.whi[1] = true; else b.yo[2] = 0; }
  if (D3) {
    if (z == 0) { if (WALLS && a.wall_z) b.wlo[2] = true; else b.zo[0] = a.nz - 1; }
    if (z == a.nz - 1) { if (WALLS && a.wall_z) b.whi[2] = true; else b.zo[2] = 0; }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b.yo[d] *= nx;
    b.zo[d] *= nxy;
  }
  // pull mask: bit k set when the population arriving along e_k comes from
  // beyond a wall face or (with solid geometry) from a solid node; one bit
  // test per direction in either case
  b.geom = false;
  b.pm = 0u;
  if (WALLS) {
    if (a.bb) {
      b.geom = true;
      b.pm = a.bb[uint32_t(x) + nx * uint32_t(y) + nxy * uint32_t(z)];
    } else {
#pragma unroll
      for (int k = 1; k < L::Q; ++k) {
        bool w = false;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (L::e[k][d] > 0) w = w || b.wlo[d];
          if (L::e[k][d] < 0) w = w || b.whi[d];
        }
        if (w) b.pm |= 1u << k;
      }
    }
  }
  return b;
}

// The population streaming into this node along e_k comes from x - e_k; if
// that node lies inside a wall it is this node's own post-collision
// population of the opposite direction (halfway bounce-back, Sec. III C).
template <class L, bool WALLS>
__device__ __forceinline__ bool pulled_from_wall(const Nbr& b, int k) {
  if (!WALLS) return false;
  return (b.pm >> k) & 1u;
}
// True when the population arriving along e_k comes from beyond a face of
// the lattice (a walled axis), open or not.
template <class L>
__device__ __forceinline__ bool crosses_face(const Nbr& b, int k) {
  bool c = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (L::e[k][d] > 0) c = c || b.wlo[d];
    if (L::e[k][d] < 0) c = c || b.whi[d];
  }
  return c;
}
// The open face (0..5 = x-, x+, y-, y+, z-, z+) the population arriving along
// e_k enters across, or -1: it crosses no face, or a wall face (a wall wins
// at a corner; between two open faces the first axis's face).  With solid
// geometry a solid node on an open face continues beyond it: if e_k without
// its component normal to the face comes from a solid node inside the
// lattice (that direction's pull bit set, no face crossed), the link is a
// wall link and -1 is returned.
template <class L, bool WALLS>
__device__ __forceinline__ int entry_face(const Nbr& b, int k, int open) {
  if (!WALLS || !open) return -1;
  int face = -1;
  bool wall = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int fc = -1;
    if (L::e[k][d] > 0 && b.wlo[d]) fc = 2 * d;
    if (L::e[k][d] < 0 && b.whi[d]) fc = 2 * d + 1;
    if (fc < 0) continue;
    if ((open >> fc) & 1) {
      if (face < 0) face = fc;
    } else {
      wall = true;
    }
  }
  if (wall) return -1;
  if (face >= 0 && b.geom) {
    bool prism = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d != (face >> 1) || L::e[k][d] == 0) continue;
      // the in-face part of e_k: e_k with component d removed
      const int kt = direction_of<L>(d == 0 ? 0 : L::e[k][0], d == 1 ? 0 : L::e[k][1], d == 2 ? 0 : L::e[k][2]);
      if (kt > 0) prism = ((b.pm >> kt) & 1u) && !crosses_face<L>(b, kt);
    }
    if (prism) return -1;
  }
  return face;
}

// Record form of f (every node relaxes with omega+ = omega- = 1): the
// post-collision f of a node is fixed by its records, Eqs. TRT, FTRT and
// hydroforce with omega = 1 giving
//   f*_k = w_k [s_k / w_k + fB + (e.F)(9/2 e.v +- 3/2)],  fB = 3 P - 3/2 v.F,
// with s_k / w_k = (e.v)(9/2 e.v +- 3) - 3/2 v.v the term the equilibrium of g
// shares, e the odd member of k's pair and + for that member.  The node
// stores (fB, F) beside its (v, -3/2 v.v).  f_scaled returns f*_k / w_k for
// direction kd from v4 = (v, -3/2 v.v) and fr = (fB, F).
template <class L, class T>
__device__ __forceinline__ T f_from_s(int kd, T ev, T u, const T (&fr)[4]) {
  const int kp = (kd & 1) ? kd : kd - 1;
  const T F[3] = {fr[1], fr[2], fr[3]};
  const T eF = proj<L>(kp, F);
  return u + fma(eF, fma(T(4.5), ev, (kd & 1) ? T(1.5) : -T(1.5)), fr[0]);
}
template <class L, class T>
__device__ __forceinline__ T f_scaled(int kd, const T (&v4)[4], const T (&fr)[4]) {
  const int kp = (kd & 1) ? kd : kd - 1;
  const T v[3] = {v4[0], v4[1], v4[2]};
  const T ev = proj<L>(kp, v);
  const T u = fma(ev, fma(T(4.5), ev, (kd & 1) ? T(3) : -T(3)), v4[3]);
  return f_from_s<L>(kd, ev, u, fr);
}
// The equilibrium of the state set_fields writes, f^eq_k(P0, v0) / w_k =
// A0 + 9/2 (e.v0)^2 +- 3 e.v0 (Eq. feq), from the record (A0, v0) with
// A0 = 3 P0 - 3/2 v0.v0.
template <class L, class T>
__device__ __forceinline__ T f_scaled_local(int kd, const T (&fr)[4]) {
  const int kp = (kd & 1) ? kd : kd - 1;
  const T v0[3] = {fr[1], fr[2], fr[3]};
  const T ev = proj<L>(kp, v0);
  const T q = fma(T(4.5) * ev, ev, fr[0]);
  return (kd & 1) ? fma(T(3), ev, q) : fma(-T(3), ev, q);
}

// Convective outflow plane: the in-plane index p of node (x, y, z) when it
// lies on the boundary plane of face `face` (inner = 1: on the plane inside
// it), else -1.  p runs over the two tangential axes, the lower one fastest.
__device__ __forceinline__ int outflow_plane_index(int face, int inner, int x, int y, int z, const StepArgs& a) {
  const int ax = face >> 1;
  const int c[3] = {x, y, z};
  const int n[3] = {a.nx, a.ny, a.nz};
  const int pos = (face & 1) ? n[ax] - 1 - inner : inner;
  if (c[ax] != pos) return -1;
  const int t0 = ax == 0 ? 1 : 0, t1 = ax == 2 ? 1 : 2;
  return c[t0] + n[t0] * c[t1];
}
__host__ __device__ __forceinline__ int outflow_plane_size(int face, int nx, int ny, int nz) {
  const int ax = face >> 1;
  const int n[3] = {nx, ny, nz};
  const int t0 = ax == 0 ? 1 : 0, t1 = ax == 2 ? 1 : 2;
  return n[t0] * n[t1];
}

// A solid node holds no fluid: the reconstruction writes C = 0 there and the
// fields read back as 0; what the update stores there is read by no fluid
// node (every pull from it is bounced back).
template <bool WALLS>
__device__ __forceinline__ bool solid_node(const Nbr& b) {
  return WALLS && b.geom && (b.pm & 1u);
}
template <class L>
__device__ __forceinline__ uint32_t upstream(const Nbr& b, int k) {
  return b.xo[1 - L::e[k][0]] + b.yo[1 - L::e[k][1]] + b.zo[1 - L::e[k][2]];
}

// Sum (op 0), max (op 1) or min (op 2) of v over a 256-thread workgroup:
// wavefront shuffles, then the four wave results through scratch[0..3] in
// LDS, in a fixed order; every thread returns the result.
__device__ __forceinline__ double block_reduce_d(double v, int op, double* scratch) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off, 64);
    v = op == 0 ? v + o : (op == 1 ? fmax(v, o) : fmin(v, o));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double r = scratch[0];
  for (int q = 1; q < 4; ++q) r = op == 0 ? r + scratch[q] : (op == 1 ? fmax(r, scratch[q]) : fmin(r, scratch[q]));
  return r;
}

// Workgroup -> tile.  Consecutive workgroup ids are dealt round-robin to the
// 8 XCDs, each with its own L2; the remap hands every XCD a contiguous run of
// tiles, so the halo rows and planes a workgroup re-reads were mostly fetched
// into the same L2 by its neighbours.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int per = nblocks >> 3;
  if (b >= per * 8) return b;
  return (b & 7) * per + (b >> 3);
}

// Typed view of a global-memory pointer of the argument structs.
template <class E>
__device__ __forceinline__ E* gptr(const NFLBM_GLOBAL void* p) {
  return (E*)(p);
}
template <class E>
__device__ __forceinline__ E* gptr(const E* p) {
  return const_cast<E*>(p);
}

// Element idx of an array addressed with a 32-bit byte offset from a uniform
// base: the load/store can then take the base in scalar registers.
template <class E>
__device__ __forceinline__ const E* at(const E* base, uint32_t idx) {
  return reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + idx * uint32_t(sizeof(E)));
}
template <class E>
__device__ __forceinline__ E* at(E* base, uint32_t idx) {
  return reinterpret_cast<E*>(reinterpret_cast<char*>(base) + idx * uint32_t(sizeof(E)));
}

// Node records of the moment form in their storage type: NV values at
// element index idx (idx * sizeof(RS) bytes from base), as values of the
// compute type (unscaled on load, scaled on store; identity for FP64 and
// FP32).  NT stores bypass the caches (streams touched once per step).
template <class S, int NV>
__device__ __forceinline__ void rec_load(const NFLBM_GLOBAL void* base, uint32_t idx, typename S::T (&o)[NV],
                                         typename S::T scale) {
  using RS = typename S::RS;
  using T = typename S::T;
  if constexpr (sizeof(RS) == sizeof(T)) {
    (void)scale;
    vld<T, NV>(at(gptr<const T>(base), idx), o);
  } else {
    RS r[NV];
    vld<RS, NV>(at(gptr<const RS>(base), idx), r);
    const T inv = T(1) / scale;
#pragma unroll
    for (int e = 0; e < NV; ++e) o[e] = static_cast<T>(r[e]) * inv;
  }
}
template <class S, int NV, bool NT>
__device__ __forceinline__ void rec_store(const NFLBM_GLOBAL void* base, uint32_t idx,
                                          const typename S::T (&v)[NV], typename S::T scale) {
  using RS = typename S::RS;
  using T = typename S::T;
  if constexpr (sizeof(RS) == sizeof(T)) {
    (void)scale;
    if constexpr (NT) vst_nt<T, NV>(at(gptr<T>(base), idx), v);
    else vst<T, NV>(at(gptr<T>(base), idx), v);
  } else {
    RS r[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) r[e] = static_cast<RS>(v[e] * scale);
    if constexpr (NT) vst_nt<RS, NV>(at(gptr<RS>(base), idx), r);
    else vst<RS, NV>(at(gptr<RS>(base), idx), r);
  }
}
// One record value (element idx).
template <class S>
__device__ __forceinline__ typename S::T rec_at(const NFLBM_GLOBAL void* base, size_t idx, typename S::T scale) {
  using RS = typename S::RS;
  using T = typename S::T;
  if constexpr (sizeof(RS) == sizeof(T)) {
    (void)scale;
    return gptr<const T>(base)[idx];
  } else {
    return static_cast<T>(gptr<const RS>(base)[idx]) / scale;
  }
}

}  // namespace nflbm
