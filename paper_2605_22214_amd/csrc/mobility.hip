// Concentration-dependent mobility (Appendix C) for gfx950.
//
// The variant replaces the constant alpha of the Cahn-Hilliard flux by the
// per-node matrix alpha_ij = C_i^2 C_j^2 (i != j), alpha_ii = -sum_{j != i}
// alpha_ij (Eq. mobilconc).  Because alpha now varies in space it is kept out
// of the gradient: g^eq carries no mobility term (m = 0 in Eq. geq) and every
// evolved g gains, after its BGK relaxation, the source of Eq. glbesource,
//   (1 - 1/(2 tau_g,i)) w_k m* e_k . G_i,   G_i = sum_j alpha_ij grad(mu_j + phi_j + xi_j),
// whose first moment drives the flux M G_i with M = c_s^2 m* (tau_g - 1/2).
//
// A step of the variant is the usual reconstruction and update (the update
// run with m = 0) with two launches around the update:
//   k_mob_potentials  after the reconstruction: Phi_j = mu_j + phi_j + xi_j
//                     for all N components at every node (Eqs. mu, G, P),
//                     from C and its Laplacian, into a scratch array;
//   k_mob_source      after the update: G_i from the isotropic gradient of Phi
//                     (Eq. gradstencil, wall neighbours replaced by the node)
//                     and the node's alpha, added to the post-collision
//                     populations the update stored at the node (pull layout:
//                     populations are stored where they were collided, so the
//                     source touches this node's values only), and the rest
//                     population re-formed as C_i minus the moving ones.
// Both are one thread per node; neighbour values come through the caches.
// An absent component has alpha_ij = 0 for every j, hence G_i = 0 and a zero
// source: it stays exactly 0.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace nflbm {

namespace {

__device__ __forceinline__ void node_xyz(uint32_t node, const StepArgs& a, int& x, int& y, int& z) {
  const uint32_t nx = a.nx, ny = a.ny;
  x = int(node % nx);
  const uint32_t r = node / nx;
  y = int(r % ny);
  z = int(r / ny);
}

// C of every component at node idx: the stored evolved ones, the implicit one
// as 1 minus their sum (in increasing component order).
template <int NC, class T>
__device__ __forceinline__ void node_conc(const T* conc, uint32_t idx, T (&c)[NC]) {
  constexpr int NE = NC - 1;
  T s[NE];
  vld<T, NE>(at(conc, idx * NE), s);
  T rest = T(0);
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    c[i] = s[i];
    rest += s[i];
  }
  c[NE] = T(1) - rest;
}

// Index of the neighbour x + e_k, or the node itself where x + e_k lies
// inside a wall (the stencil rule of the wall paragraph of Sec. III C).
// x + e_k is the upstream node of the opposite direction.
template <class L, bool WALLS>
__device__ __forceinline__ uint32_t stencil_node(const Nbr& b, int k, uint32_t node) {
  const int kb = opposite(k);
  return pulled_from_wall<L, WALLS>(b, kb) ? node : upstream<L>(b, kb);
}

}  // namespace

// Phi_j = mu_j + phi_j + xi_j of every component j at every node:
//   mu_j  = sum_{k != j} [beta_jk (f'(C_j) - f'(C_j + C_k))] + sum_{k != j} kappa_jk lap C_k
//   phi_j = (12/D) sum_{k<l<m, none j} Lambda_{j;klm} C_k C_l C_m
//   xi_j  = (12/D) Omega sum_{k<l, none j} C_k^2 C_l^2 (2 C_j - sum_{m not in jkl} Theta_{kl;j;m} C_m)
// with lap C = (2/c_s^2) sum_{k>=1} w_k [C(x + e_k) - C(x)].
template <class L, int NC, class T, bool WALLS>
__global__ void __launch_bounds__(256) k_mob_potentials(MobArgs ma) {
  const StepArgs& a = ma.sa;
  const uint32_t node = blockIdx.x * 256u + threadIdx.x;
  if (node >= uint32_t(a.n)) return;
  const DevParams<T>& P = *gptr<const DevParams<T>>(a.params);
  const MobParams<T>& M = *static_cast<const MobParams<T>*>(ma.mob);
  const T* conc = gptr<const T>(a.conc);
  int x, y, z;
  node_xyz(node, a, x, y, z);
  const Nbr nb = neighbours<L, WALLS>(x, y, z, a);
  T c[NC];
  node_conc<NC, T>(conc, node, c);
  T lap[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) lap[j] = T(0);
#pragma unroll
  for (int k = 1; k < L::Q; ++k) {
    T cn[NC];
    node_conc<NC, T>(conc, stencil_node<L, WALLS>(nb, k, node), cn);
    const T wk = static_cast<T>(L::w[k]);
#pragma unroll
    for (int j = 0; j < NC; ++j) lap[j] = fma(wk, cn[j] - c[j], lap[j]);
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) lap[j] *= T(6);

  T phi_out[NC];
  const bool omega = (a.flags & kFlagOmega) != 0;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    T mu = T(0);
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k != j) mu = fma(P.beta[j][k], fprime(c[j]) - fprime(c[j] + c[k]), mu);
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k != j) mu = fma(P.kappa[j][k], lap[k], mu);
    T ph = T(0);
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int l = k + 1; l < NC; ++l)
#pragma unroll
        for (int m = l + 1; m < NC; ++m)
          if (k != j && l != j && m != j) ph = fma(M.lam[j][k][l][m], c[k] * c[l] * c[m], ph);
    T xi = T(0);
    if (omega) {
#pragma unroll
      for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = k + 1; l < NC; ++l) {
          if (k == j || l == j) continue;
          T inner = T(2) * c[j];
#pragma unroll
          for (int m = 0; m < NC; ++m)
            if (m != j && m != k && m != l) inner = fma(-M.theta[k][l][j][m], c[m], inner);
          xi = fma((c[k] * c[k]) * (c[l] * c[l]), inner, xi);
        }
      xi *= P.k12D * P.omega_stab;
    }
    phi_out[j] = fma(P.k12D, ph, mu) + xi;
  }
  vst<T, NC>(at(static_cast<T*>(ma.phi), node * NC), phi_out);
}

// G_i = sum_j alpha_ij(C) grad Phi_j, grad psi = (1/c_s^2) sum_{k>=1} w_k e_k
// [psi(x + e_k) - psi(x)], and the source (1 - 1/(2 tau_g,i)) w_k m* e_k.G_i
// added to the post-collision moving populations of every evolved component
// stored at this node; the rest population becomes C_i minus their sum.
template <class L, int NC, int ST, bool WALLS>
__global__ void __launch_bounds__(256) k_mob_source(MobArgs ma) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  constexpr int NE = NC - 1;
  const StepArgs& a = ma.sa;
  const uint32_t node = blockIdx.x * 256u + threadIdx.x;
  if (node >= uint32_t(a.n)) return;
  const MobParams<T>& M = *static_cast<const MobParams<T>*>(ma.mob);
  const T* phi = static_cast<const T*>(ma.phi);
  int x, y, z;
  node_xyz(node, a, x, y, z);
  const Nbr nb = neighbours<L, WALLS>(x, y, z, a);
  T p0[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) p0[j] = phi[size_t(node) * NC + j];
  T grad[NC][3];
#pragma unroll
  for (int j = 0; j < NC; ++j) grad[j][0] = grad[j][1] = grad[j][2] = T(0);
#pragma unroll
  for (int k = 1; k < L::Q; ++k) {
    const uint32_t q = stencil_node<L, WALLS>(nb, k, node);
    const T wk = static_cast<T>(L::w[k]);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const T d = wk * (phi[size_t(q) * NC + j] - p0[j]);
#pragma unroll
      for (int e = 0; e < 3; ++e)
        if (L::e[k][e] != 0) grad[j][e] = (L::e[k][e] > 0) ? grad[j][e] + d : grad[j][e] - d;
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j)
#pragma unroll
    for (int e = 0; e < 3; ++e) grad[j][e] *= T(3);

  T c[NC];
  node_conc<NC, T>(gptr<const T>(a.conc), node, c);
  T c2[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) c2[j] = c[j] * c[j];
  // pre_i G_i for the evolved components
  T G[NE][3];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    T aii = T(0);
    T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j == i) continue;
      const T aij = c2[i] * c2[j];
      aii -= aij;
#pragma unroll
      for (int e = 0; e < 3; ++e) acc[e] = fma(aij, grad[j][e], acc[e]);
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) G[i][e] = M.pre[i] * fma(aii, grad[i][e], acc[e]);
  }

  FS* gk = gptr<FS>(a.gk_dst);
  T moved[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) moved[i] = T(0);
#pragma unroll
  for (int k = 1; k < L::Q; ++k) {
    FS* p = at(gk + size_t(k - 1) * size_t(a.gstride), node * NE);
    FS v[NE];
    vld<FS, NE>(p, v);
    const T wk = static_cast<T>(L::w[k]);
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const T eG = proj<L>(k, G[i]);
      v[i] = S::pack(S::unpack(v[i]) + wk * eG);
      moved[i] += S::unpack(v[i]);
    }
    vst<FS, NE>(p, v);
  }
  G0S r0[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) r0[i] = static_cast<G0S>(c[i] - moved[i]);
  vst<G0S, NE>(at(gptr<G0S>(a.g0_dst), node * NE), r0);
}

namespace {

#define NFLBM_MOB_NC_SWITCH(NCV, CALL)    \
  switch (NCV) {                          \
    case 2: return CALL(2);               \
    case 3: return CALL(3);               \
    case 4: return CALL(4);               \
    case 5: return CALL(5);               \
    case 6: return CALL(6);               \
    case 7: return CALL(7);               \
    case 8: return CALL(8);               \
    default: return hipErrorInvalidValue; \
  }

inline bool walls_of(const StepArgs& a) { return a.wall_x || a.wall_y || a.wall_z || a.bb != nullptr; }
inline dim3 node_grid(const StepArgs& a) { return dim3(static_cast<unsigned>((a.n + 255) / 256)); }

template <class L, int NC, class T>
hipError_t potentials_t(const MobArgs& a, hipStream_t s) {
  if (walls_of(a.sa)) hipLaunchKernelGGL((k_mob_potentials<L, NC, T, true>), node_grid(a.sa), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_mob_potentials<L, NC, T, false>), node_grid(a.sa), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <class L, int NC, int ST>
hipError_t source_t(const MobArgs& a, hipStream_t s) {
  if (walls_of(a.sa)) hipLaunchKernelGGL((k_mob_source<L, NC, ST, true>), node_grid(a.sa), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_mob_source<L, NC, ST, false>), node_grid(a.sa), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <class L, class T>
hipError_t potentials_nc(int nc, const MobArgs& a, hipStream_t s) {
#define CALL_P(K) potentials_t<L, K, T>(a, s)
  NFLBM_MOB_NC_SWITCH(nc, CALL_P)
#undef CALL_P
}

template <class L, int ST>
hipError_t source_nc(int nc, const MobArgs& a, hipStream_t s) {
#define CALL_S(K) source_t<L, K, ST>(a, s)
  NFLBM_MOB_NC_SWITCH(nc, CALL_S)
#undef CALL_S
}

template <int ST>
hipError_t source_st(int lat, int nc, const MobArgs& a, hipStream_t s) {
  return lat == 0 ? source_nc<D2Q9, ST>(nc, a, s) : source_nc<D3Q19, ST>(nc, a, s);
}

}  // namespace

hipError_t launch_mob_potentials(int lat, int nc, int store, const MobArgs& a, hipStream_t s) {
  if (store == kStoreF64)
    return lat == 0 ? potentials_nc<D2Q9, double>(nc, a, s) : potentials_nc<D3Q19, double>(nc, a, s);
  return lat == 0 ? potentials_nc<D2Q9, float>(nc, a, s) : potentials_nc<D3Q19, float>(nc, a, s);
}

hipError_t launch_mob_source(int lat, int nc, int store, const MobArgs& a, hipStream_t s) {
  switch (store) {
    case kStoreF64: return source_st<kStoreF64>(lat, nc, a, s);
    case kStoreF32: return source_st<kStoreF32>(lat, nc, a, s);
    case kStoreF16S: return source_st<kStoreF16S>(lat, nc, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace nflbm
