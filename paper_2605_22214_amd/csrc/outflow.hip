// Convective outflow (Sec. III C, Eq. convect) for gfx950.
//
// On an outflow face every population of the boundary plane (plane N) is
// replaced after streaming by
//   q(N, t+1) = (q(N, t) + U q(N-1, t+1)) / (1 + U),
// q(N, t) the plane's post-streaming values of the previous step and U the
// mean over plane N-1 of the normal momentum sum_k (e_k . n) f_k after
// streaming (n the outward normal; U = 0 where that mean points inwards).
// Stencil neighbours beyond the face read ghost values of C_i and E_B that are
// convected the same way, psi(N+1, t+1) = (psi(N+1, t) + U psi(N, t+1)) /
// (1 + U), from psi(N, 0).
//
// The state holds post-collision populations (pull streaming), so the
// post-streaming values of plane N have no place in it: they live in a plane
// buffer of their own (out_f, out_g, every direction including the rest one),
// which the reconstruction and the update read at plane-N nodes in place of
// their pulls, and the update's LDS fill reads the ghost buffer beyond the
// face.  Per step, after the update (on the state it wrote), both kernels
// with 64 plane nodes per workgroup and each node's directions split over
// the workgroup's eight wavefronts (two per SIMD, so that the gathers across
// the face overlap):
//   k_outflow_mom    the normal momentum of plane N-1 after streaming,
//                    gathered with the pull rules of the update; one FP64
//                    sum per workgroup;
//   k_outflow_apply  every workgroup sums those partial sums in one fixed
//                    order (so all of them hold the same U), then blends the
//                    pulled plane N-1 populations into the plane buffer and
//                    convects the ghosts.
// With start = 1 the apply kernel instead captures plane N of the current
// state (q(N, 0), ghosts C(N, 0) and E_B(N, 0)); with start = 2 it only
// re-derives plane N's C, E_B and f moments from the buffers (after a state
// is restored).  In the moment form the reconstruction leaves the boundary
// plane to this kernel, which writes those where the reconstruction writes.
// Solid nodes continue straight through the outflow plane: U is the mean
// over the fluid nodes of plane N-1, and solid plane nodes keep zeros.  In
// the moment form of g (and the record form of f) the pulled populations are
// formed from the source nodes' records, as the reconstruction forms them.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device.h"

namespace nflbm {

namespace {

// Coordinates of in-plane index p on plane `pos` of axis `ax` (the inverse of
// outflow_plane_index).
__device__ __forceinline__ void plane_node(int ax, int pos, int p, const StepArgs& a, int& x, int& y, int& z) {
  const int n[3] = {a.nx, a.ny, a.nz};
  const int t0 = ax == 0 ? 1 : 0, t1 = ax == 2 ? 1 : 2;
  int c[3];
  c[ax] = pos;
  c[t0] = p % n[t0];
  c[t1] = p / n[t0];
  x = c[0];
  y = c[1];
  z = c[2];
}

__device__ __forceinline__ int plane_pos(int face, int inner, const StepArgs& a) {
  const int ax = face >> 1;
  const int n = ax == 0 ? a.nx : (ax == 1 ? a.ny : a.nz);
  return (face & 1) ? n - 1 - inner : inner;
}

// Post-collision f*_kd of the node at index src in the record form of f:
// w_kd times f_scaled of its records (v, -3/2 v.v) and (fB, F).
template <class L, int ST>
__device__ __forceinline__ typename StoreT<ST>::T rec_f(const StepArgs& a, uint32_t src, int kd) {
  using S = StoreT<ST>;
  using T = typename S::T;
  T v4[4], fr[4];
  rec_load<S, 4>(a.vel, src * 4u, v4, T(S::vel_scale));
  rec_load<S, 4>(a.frec, src * 4u, fr, T(S::vel_scale));
  return static_cast<T>(L::w[kd]) * f_scaled<L>(kd, v4, fr);
}
// Post-streaming f_k (k >= 1) of a node, pulled as the update pulls it:
// halfway bounce-back at a wall face, plus the velocity correction where the
// link enters across an open face.  In the record form of f the
// post-collision values are formed from the source's records (on the first
// step after set_fields: the node's own initial equilibrium).
template <class L, int ST>
__device__ __forceinline__ typename StoreT<ST>::T pull_f(const StepArgs& a, const Nbr& nb, uint32_t node, int k,
                                                         const FaceBC<typename StoreT<ST>::T>* FB, int open) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  if (a.flags & kFlagFRecord) {
    if (a.flags & kFlagFLocal) {
      T fr[4];
      rec_load<S, 4>(a.frec, node * 4u, fr, T(S::vel_scale));
      return static_cast<T>(L::w[k]) * f_scaled_local<L>(k, fr);
    }
    if (pulled_from_wall<L, true>(nb, k)) {
      T v = rec_f<L, ST>(a, node, opposite(k));
      const int fc = entry_face<L, true>(nb, k, open);
      if (fc >= 0) v += FB->fcorr[fc][k];
      return v;
    }
    return rec_f<L, ST>(a, upstream<L>(nb, k), k);
  }
  const FS* fs = gptr<const FS>(a.f_src);
  const size_t fst = static_cast<size_t>(a.fstride);
  if (pulled_from_wall<L, true>(nb, k)) {
    T v = S::ld(fs + size_t(opposite(k) - 1) * fst, node);
    const int fc = entry_face<L, true>(nb, k, open);
    if (fc >= 0) v += FB->fcorr[fc][k];
    return v;
  }
  return S::ld(fs + size_t(k - 1) * fst, upstream<L>(nb, k));
}

// Post-streaming g_{e,k} (any k) of every evolved component e, pulled as the
// reconstruction pulls them (anti-bounce-back across an open face), the
// source's record (or populations) read once for all components.  In the
// moment form the post-collision values are formed from the records: g*_k =
// C_e s_k(v) - w_k m mu~_e (Eq. geq with tau_g = 1), the rest population
// C_e (1 + s_0) + (1 - w_0) m mu~_e of the node's own; on the first step
// after set_fields g entering across an open face is the initial 0.
template <class L, int NE, int ST>
__device__ __forceinline__ void pull_g_all(const StepArgs& a, const Nbr& nb, uint32_t node, int k,
                                           const FaceBC<typename StoreT<ST>::T>* FB, int open,
                                           typename StoreT<ST>::T (&q)[NE]) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  if (a.flags & kFlagMoments) {
    const DevParams<T>& P = *gptr<const DevParams<T>>(a.params);
    T c[NE], mu[NE], v4[4];
    const bool wall = k > 0 && pulled_from_wall<L, true>(nb, k);
    const uint32_t src = (k == 0 || wall) ? node : upstream<L>(nb, k);
    vld<T, NE>(gptr<const T>(a.cprev) + size_t(src) * NE, c);
    rec_load<S, NE>(a.mu, src * uint32_t(NE), mu, T(S::mu_scale));
    rec_load<S, 4>(a.vel, src * 4u, v4, T(S::vel_scale));
    if (k == 0) {
      const T s0 = static_cast<T>(L::w[0]) * v4[3];
#pragma unroll
      for (int e = 0; e < NE; ++e) q[e] = c[e] + fma(c[e], s0, (static_cast<T>(1.0 - L::w[0]) * P.m) * mu[e]);
      return;
    }
    const int kd = wall ? opposite(k) : k;
    const int kp = (kd & 1) ? kd : kd - 1;
    const T v[3] = {v4[0], v4[1], v4[2]};
    const T ev = proj<L>(kp, v);
    const T u = fma(ev, fma(T(4.5), ev, (kd & 1) ? T(3) : -T(3)), v4[3]);
    const T wk = static_cast<T>(L::w[kd]);
#pragma unroll
    for (int e = 0; e < NE; ++e) q[e] = fma(c[e], wk * u, -(wk * P.m) * mu[e]);
    if (wall) {
      const int fc = entry_face<L, true>(nb, k, open);
      if (fc >= 0) {
#pragma unroll
        for (int e = 0; e < NE; ++e) q[e] = (a.flags & kFlagFLocal) ? T(0) : FB->gsum[fc][e][k] - q[e];
      }
    }
    return;
  }
  if (k == 0) {
    G0S r[NE];
    vld<G0S, NE>(gptr<const G0S>(a.g0_src) + size_t(node) * NE, r);
#pragma unroll
    for (int e = 0; e < NE; ++e) q[e] = static_cast<T>(r[e]);
    return;
  }
  const FS* gk = gptr<const FS>(a.gk_src);
  const size_t gst = static_cast<size_t>(a.gstride);
  FS r[NE];
  if (pulled_from_wall<L, true>(nb, k)) {
    vld<FS, NE>(gk + size_t(opposite(k) - 1) * gst + size_t(node) * NE, r);
    const int fc = entry_face<L, true>(nb, k, open);
#pragma unroll
    for (int e = 0; e < NE; ++e) q[e] = fc >= 0 ? FB->gsum[fc][e][k] - S::unpack(r[e]) : S::unpack(r[e]);
    return;
  }
  vld<FS, NE>(gk + size_t(k - 1) * gst + size_t(upstream<L>(nb, k)) * NE, r);
#pragma unroll
  for (int e = 0; e < NE; ++e) q[e] = S::unpack(r[e]);
}

}  // namespace

// Work split of both kernels: a workgroup takes kOutNodes plane nodes (one
// per lane) and its kOutWaves wavefronts take the directions of those nodes
// in turn, wavefront w the directions k = w, w + kOutWaves, ...  Each wave
// sums its directions in that order; the workgroup then adds the waves'
// partial sums in wave order, so every result has one fixed order.
constexpr int kOutWaves = kOutThreads / kOutNodes;

// Runs f(std::integral_constant<int, w>) for the wave index w of this thread,
// so that a wave's direction loop has compile-time directions.
template <class F>
__device__ __forceinline__ void for_wave(int w, F&& f) {
  static_assert(kOutWaves == 8, "eight direction groups per workgroup");
  switch (w) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    default: f(std::integral_constant<int, 7>{}); break;
  }
}

template <class L, int NC, int ST>
__global__ void __launch_bounds__(kOutThreads) k_outflow_mom(OutflowArgs o) {
  using T = typename StoreT<ST>::T;
  const StepArgs& a = o.sa;
  __shared__ double red[kOutThreads];
  const int face = a.out_face, ax = face >> 1;
  const double sgn = (face & 1) ? 1.0 : -1.0;      // outward normal along ax
  const int PL = outflow_plane_size(face, a.nx, a.ny, a.nz);
  const int lane = static_cast<int>(threadIdx.x) % kOutNodes;
  const int wave = static_cast<int>(threadIdx.x) / kOutNodes;
  const int p = static_cast<int>(blockIdx.x) * kOutNodes + lane;
  double mom = 0.0;
  if (p < PL) {
    int x, y, z;
    plane_node(ax, plane_pos(face, 1, a), p, a, x, y, z);
    const Nbr nb = neighbours<L, true>(x, y, z, a);
    const uint32_t node = uint32_t(x) + uint32_t(a.nx) * (uint32_t(y) + uint32_t(a.ny) * uint32_t(z));
    const FaceBC<T>* FB = gptr<const FaceBC<T>>(a.faces);
    const int open = FB ? FB->open : 0;
    if (!solid_node<true>(nb)) {       // solid nodes hold no fluid
      for_wave(wave, [&](auto WC) {
        constexpr int W = decltype(WC)::value;
#pragma unroll
        for (int k = (W == 0 ? kOutWaves : W); k < L::Q; k += kOutWaves) {
          if (L::e[k][ax] == 0) continue;
          const double v = static_cast<double>(pull_f<L, ST>(a, nb, node, k, FB, open));
          mom += (L::e[k][ax] > 0) ? v : -v;
        }
      });
      mom *= sgn;
    }
  }
  red[threadIdx.x] = mom;
  __syncthreads();
  for (int s = kOutThreads / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) o.partial[blockIdx.x] = red[0];
}

template <class L, int NC, int ST>
__global__ void __launch_bounds__(kOutThreads) k_outflow_apply(OutflowArgs o) {
  using S = StoreT<ST>;
  using T = typename S::T;
  constexpr int NE = NC - 1;
  constexpr int Q = L::Q;
  constexpr int NPART = NE + 4;        // per wave and node: sum of moving g, f moments
  const StepArgs& a = o.sa;
  __shared__ double red[kOutThreads];
  __shared__ T part[kOutWaves][NPART][kOutNodes];
  const int face = a.out_face, ax = face >> 1;
  const int PL = outflow_plane_size(face, a.nx, a.ny, a.nz);
  const int tid = static_cast<int>(threadIdx.x);
  const int lane = tid % kOutNodes;
  const int wave = tid / kOutNodes;
  // U from the partial sums, in the same order in every workgroup
  double U = 0.0;
  if (o.start == 0) {
    double s = 0.0;
    for (int i = tid; i < o.blocks; i += kOutThreads) s += o.partial[i];
    red[tid] = s;
    __syncthreads();
    for (int w = kOutThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    U = red[0] / o.fluid;          // mean over the fluid nodes of plane N-1
    if (!(U > 0.0)) U = 0.0;
    if (blockIdx.x == 0 && tid == 0) o.u[0] = U;
  }
  const int p = static_cast<int>(blockIdx.x) * kOutNodes + lane;
  const bool active = p < PL;
  const size_t P = static_cast<size_t>(PL);
  T* of = gptr<T>(a.out_f);
  T* og = gptr<T>(a.out_g);
  T* gh = gptr<T>(a.out_ghost);
  // plane N's node (the boundary plane) and, for convecting, plane N-1's
  int xN = 0, yN = 0, zN = 0;
  if (active) plane_node(ax, plane_pos(face, 0, a), p, a, xN, yN, zN);
  const uint32_t nodeN = uint32_t(xN) + uint32_t(a.nx) * (uint32_t(yN) + uint32_t(a.ny) * uint32_t(zN));
  bool solid = false;
  if (active) solid = solid_node<true>(neighbours<L, true>(xN, yN, zN, a));
  const bool moments = (a.flags & kFlagMoments) != 0;
  if (o.start == 2 && !moments) return;          // nothing to refresh
  // this wave's directions: blend (start 0), capture (start 1) or only read
  // back (start 2) their plane-N values, and sum them per node
  T m[NE], r[NE], fm[4];
#pragma unroll
  for (int e = 0; e < NE; ++e) m[e] = r[e] = T(0);
#pragma unroll
  for (int d = 0; d < 4; ++d) fm[d] = T(0);
  if (active && !solid) {
    int x, y, z;
    plane_node(ax, plane_pos(face, o.start == 0 ? 1 : 0, a), p, a, x, y, z);
    const Nbr nb = neighbours<L, true>(x, y, z, a);
    const uint32_t node = uint32_t(x) + uint32_t(a.nx) * (uint32_t(y) + uint32_t(a.ny) * uint32_t(z));
    const FaceBC<T>* FB = gptr<const FaceBC<T>>(a.faces);
    const int open = FB ? FB->open : 0;
    const T u = static_cast<T>(U);
    const T den = T(1) + u;
    for_wave(wave, [&](auto WC) {
      constexpr int W = decltype(WC)::value;
#pragma unroll
      for (int k = W; k < Q; k += kOutWaves) {
        if (k >= 1) {
          T* slot = of + size_t(k - 1) * P + p;
          T v;
          if (o.start == 2) {
            v = *slot;
          } else {
            const T q = pull_f<L, ST>(a, nb, node, k, FB, open);
            v = o.start ? q : (*slot + u * q) / den;
            *slot = v;
          }
          fm[0] += v;
#pragma unroll
          for (int d = 0; d < 3; ++d)
            if (L::e[k][d] != 0) fm[1 + d] += (L::e[k][d] > 0) ? v : -v;
        }
        T q[NE];
        if (o.start != 2) pull_g_all<L, NE, ST>(a, nb, node, k, FB, open, q);
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          T* slot = og + (size_t(e) * Q + k) * P + p;
          T v;
          if (o.start == 2) {
            v = *slot;
          } else {
            v = o.start ? q[e] : (*slot + u * q[e]) / den;
            *slot = v;
          }
          if (k == 0) r[e] = v;
          else m[e] += v;
        }
      }
    });
  } else if (active && o.start != 2) {
    // a solid node of the plane (solid nodes continue straight through the
    // outflow plane, so plane N-1 is solid here too): no fluid
    for_wave(wave, [&](auto WC) {
      constexpr int W = decltype(WC)::value;
#pragma unroll
      for (int k = W; k < Q; k += kOutWaves) {
        if (k >= 1) of[size_t(k - 1) * P + p] = T(0);
#pragma unroll
        for (int e = 0; e < NE; ++e) og[(size_t(e) * Q + k) * P + p] = T(0);
      }
    });
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) part[wave][e][lane] = m[e];
#pragma unroll
  for (int d = 0; d < 4; ++d) part[wave][NE + d][lane] = fm[d];
  __syncthreads();
  if (wave != 0 || !active) return;
  if (solid) {
    // a stencil never reads a solid node's ghost (the solid continues beyond
    // the face)
    if (o.start != 2)
      for (int e = 0; e <= NE; ++e) gh[size_t(e) * P + p] = T(0);
    return;
  }
  // C as the reconstruction sums it: the moving populations, then the rest
  T c[NC];
  T rest = T(0);
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    T mt = part[0][e][lane];
#pragma unroll
    for (int w = 1; w < kOutWaves; ++w) mt += part[w][e][lane];
    c[e] = r[e] + mt;
    rest += c[e];
  }
  c[NE] = T(1) - rest;
  const DevParams<T>& Pp = *gptr<const DevParams<T>>(a.params);
  const T E = bulk_energy<NC, T>(c, Pp);
  if (o.start != 2) {
    const T u = static_cast<T>(U);
    const T den = T(1) + u;
    for (int e = 0; e < NE; ++e) {
      T* slot = gh + size_t(e) * P + p;
      *slot = o.start ? c[e] : (*slot + u * c[e]) / den;
    }
    T* slot = gh + size_t(NE) * P + p;
    *slot = o.start ? E : (*slot + u * E) / den;
  }
  if (moments) {
    // In the moment form the next reconstruction leaves the boundary plane
    // to this kernel: C, E_B and (record form of f) the f moments of the new
    // plane-N populations, where that reconstruction writes its results
    vst<T, NE>(gptr<T>(a.conc) + size_t(nodeN) * NE, reinterpret_cast<const T(&)[NE]>(c));
    gptr<T>(a.eb)[nodeN] = E;
    if (a.flags & kFlagFRecord) {
      T ft[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        ft[d] = part[0][NE + d][lane];
#pragma unroll
        for (int w = 1; w < kOutWaves; ++w) ft[d] += part[w][NE + d][lane];
      }
      rec_store<S, 4, false>(a.fmom, nodeN * 4u, ft, T(S::vel_scale));
    }
  }
}

namespace {

#define NFLBM_OUT_NC_SWITCH(NCV, CALL)    \
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

template <class L, int NC, int ST>
hipError_t outflow_t(const OutflowArgs& o, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(o.blocks));   // kOutNodes plane nodes each
  if (o.start == 0) hipLaunchKernelGGL((k_outflow_mom<L, NC, ST>), grid, dim3(kOutThreads), 0, s, o);
  hipLaunchKernelGGL((k_outflow_apply<L, NC, ST>), grid, dim3(kOutThreads), 0, s, o);
  return hipGetLastError();
}

template <class L, int ST>
hipError_t outflow_nc(int nc, const OutflowArgs& o, hipStream_t s) {
#define CALL_O(K) outflow_t<L, K, ST>(o, s)
  NFLBM_OUT_NC_SWITCH(nc, CALL_O)
#undef CALL_O
}

template <int ST>
hipError_t outflow_st(int lat, int nc, const OutflowArgs& o, hipStream_t s) {
  return lat == 0 ? outflow_nc<D2Q9, ST>(nc, o, s) : outflow_nc<D3Q19, ST>(nc, o, s);
}

}  // namespace

hipError_t launch_outflow(int lat, int nc, int store, const OutflowArgs& o, hipStream_t s) {
  if (o.sa.out_face < 0 || o.blocks < 1) return hipErrorInvalidValue;
  switch (store) {
    case kStoreF64: return outflow_st<kStoreF64>(lat, nc, o, s);
    case kStoreF32: return outflow_st<kStoreF32>(lat, nc, o, s);
    case kStoreF16S: return outflow_st<kStoreF16S>(lat, nc, o, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace nflbm
