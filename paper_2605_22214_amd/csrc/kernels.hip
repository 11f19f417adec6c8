// Device code of the N-component free-energy LBM time step for gfx950.
//
// One time step = two launches:
//   k_conc    C_i = sum_k g_{i,k} for the evolved components (zeroth moment
//             of g, Sec. III B).  Reads every g population once, writes NE
//             values per node.
//   k_update  per node: C of all components from an LDS halo tile (the
//             implicit one as 1 - sum of the others), E_B, the isotropic
//             gradient/Laplacian stencils (Eq. gradstencil) with the wall
//             rule, the flux potential mu~ in factored form, the conservative
//             surface-tension force (Eq. Fsnew), v and P (Eqs. nmom, pres),
//             node viscosity, TRT collision with forcing (Eqs. TRT, FTRT,
//             hydroforce), BGK collision of g (Eq. glbe), push streaming with
//             halfway bounce-back.  Reads f once, writes f and g once.
// The concentration equilibrium is the rest-population form
//   g^eq_{i,0} = C_i (1 + s_0) + (1 - w_0) m mu~_i,  g^eq_{i,k} = C_i s_k - w_k m mu~_i;
// the rest population is written as C_i minus the stored moving populations,
// which equals g^eq_{i,0} in exact arithmetic and keeps node mass to the
// rounding of one value in every storage precision.
//
// Workgroups are 256 threads covering a TX x TY tile of the x-y plane.  The
// D2Q9 kernel loads one LDS plane; the D3Q19 kernel marches along z through
// zchunk planes with a rolling window of three LDS planes.
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

// ----------------------------------------------------------- storage types
template <int ST> struct StoreT;
template <> struct StoreT<kStoreF64> {
  using T = double; using FS = double; using G0S = double;
  static __device__ __forceinline__ T ld(const FS* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ FS pack(T v) { return v; }
  static __device__ __forceinline__ T unpack(FS v) { return v; }
};
template <> struct StoreT<kStoreF32> {
  using T = float; using FS = float; using G0S = float;
  static __device__ __forceinline__ T ld(const FS* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ FS pack(T v) { return v; }
  static __device__ __forceinline__ T unpack(FS v) { return v; }
};
template <> struct StoreT<kStoreF16S> {
  using T = float; using FS = _Float16; using G0S = float;
  static __device__ __forceinline__ T ld(const FS* p, size_t i) {
    return static_cast<float>(p[i]) * (1.0f / kHalfScale);
  }
  static __device__ __forceinline__ FS pack(T v) { return static_cast<_Float16>(v * kHalfScale); }
  static __device__ __forceinline__ T unpack(FS v) { return static_cast<float>(v) * (1.0f / kHalfScale); }
};

template <class T>
__device__ __forceinline__ T fpoly(T c) {
  const T d = T(1) - c;
  return c * c * d * d;
}
template <class T>
__device__ __forceinline__ T fprime(T c) {
  return T(2) * c * (T(1) - T(3) * c + T(2) * c * c);
}

// E_B = sum_{i<j} beta_ij [f(C_i) + f(C_j) - f(C_i + C_j)]  (Eq. FreeEnergy)
template <int NC, class T>
__device__ __forceinline__ T bulk_energy(const T (&c)[NC], const DevParams<T>& P) {
  T fi[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) fi[i] = fpoly(c[i]);
  T e = T(0);
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = i + 1; j < NC; ++j) e += P.beta[i][j] * (fi[i] + fi[j] - fpoly(c[i] + c[j]));
  return e;
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ------------------------------------------------------------------ k_conc
template <int Q, int ST>
__global__ void __launch_bounds__(256) k_conc(StepArgs a, int ne) {
  using S = StoreT<ST>;
  using T = typename S::T;
  const typename S::G0S* g0 = static_cast<const typename S::G0S*>(a.g0_src);
  const typename S::FS* gk = static_cast<const typename S::FS*>(a.gk_src);
  T* C = static_cast<T*>(a.conc);
  const size_t n = static_cast<size_t>(a.n);
  for (size_t node = blockIdx.x * size_t(256) + threadIdx.x; node < n;
       node += size_t(gridDim.x) * 256) {
    for (int e = 0; e < ne; ++e) {
      T s = static_cast<T>(g0[e * n + node]);
      const typename S::FS* base = gk + size_t(e) * (Q - 1) * n + node;
#pragma unroll
      for (int k = 0; k < Q - 1; ++k) s += S::ld(base, size_t(k) * n);
      C[e * n + node] = s;
    }
  }
}

// ---------------------------------------------------------------- k_update
template <class L, int NC, int ST, bool FIELDS>
__global__ void __launch_bounds__(256) k_update(StepArgs a) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  constexpr int Q = L::Q;
  constexpr int NE = NC - 1;
  constexpr int NPL = (L::DIM == 3) ? 3 : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const DevParams<T>& P = *static_cast<const DevParams<T>*>(a.params);

  const int tid = threadIdx.x;
  const int TX = 1 << a.tx_log2;
  const int TY = 256 >> a.tx_log2;
  const int tx = tid & (TX - 1);
  const int ty = tid >> a.tx_log2;
  const int PX = TX + 2;
  const int PXY = PX * (TY + 2);
  const int plane_stride = (NE + 1) * PXY;

  int b = blockIdx.x;
  const int tile_x = b % a.tiles_x;
  b /= a.tiles_x;
  const int tile_y = b % a.tiles_y;
  const int chunk = b / a.tiles_y;
  const int x0 = tile_x * TX, y0 = tile_y * TY;
  const int z0 = chunk * a.zchunk;
  const int z1 = min(z0 + a.zchunk, a.nz);
  const int x = x0 + tx, y = y0 + ty;
  const bool active = (x < a.nx) && (y < a.ny);
  const size_t n = static_cast<size_t>(a.n);
  const T* conc = static_cast<const T*>(a.conc);

  // Fill LDS slot with C (evolved components) and E_B for plane gz, tile plus
  // a one-node ring.  Positions inside a wall are not filled: the stencil
  // never reads them.
  auto load_plane = [&](int slot, int gz) {
    T* base = sm + slot * plane_stride;
    bool zok = true;
    if (gz < 0 || gz >= a.nz) {
      if (a.wall_z) zok = false;
      else gz = wrap(gz, a.nz);
    }
    for (int idx = tid; idx < PXY; idx += 256) {
      const int ly = idx / PX;
      const int lx = idx - ly * PX;
      int gx = x0 + lx - 1, gy = y0 + ly - 1;
      bool ok = zok;
      if (gx < 0 || gx >= a.nx) {
        if (a.wall_x) ok = false;
        else gx = wrap(gx, a.nx);
      }
      if (gy < 0 || gy >= a.ny) {
        if (a.wall_y) ok = false;
        else gy = wrap(gy, a.ny);
      }
      if (!ok) continue;
      const size_t node = size_t(gx) + size_t(a.nx) * (size_t(gy) + size_t(a.ny) * size_t(gz));
      T c[NC];
      T rest = T(0);
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        c[e] = conc[e * n + node];
        rest += c[e];
        base[e * PXY + idx] = c[e];
      }
      c[NE] = T(1) - rest;
      base[NE * PXY + idx] = bulk_energy<NC, T>(c, P);
    }
  };

  auto process = [&](int z, int s_dn, int s_c, int s_up) {
    const int li = (ty + 1) * PX + (tx + 1);
    const T* Cc = sm + s_c * plane_stride;
    T c[NC];
    {
      T rest = T(0);
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        c[e] = Cc[e * PXY + li];
        rest += c[e];
      }
      c[NE] = T(1) - rest;
    }
    const T E0 = Cc[NE * PXY + li];
    T gC[NC][3];
    T lap[NC];
    T gE[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      lap[i] = T(0);
      gC[i][0] = gC[i][1] = gC[i][2] = T(0);
    }
    // ---- isotropic stencils (Eq. gradstencil and the Laplacian after it)
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const int ex = L::e[k][0], ey = L::e[k][1], ez = L::e[k][2];
      const T wk = static_cast<T>(L::w[k]);
      bool wall = false;
      if (ex != 0 && a.wall_x) wall |= (x + ex < 0) || (x + ex >= a.nx);
      if (ey != 0 && a.wall_y) wall |= (y + ey < 0) || (y + ey >= a.ny);
      if (ez != 0 && a.wall_z) wall |= (z + ez < 0) || (z + ez >= a.nz);
      if (!wall) {
        const int slot = (ez == 0) ? s_c : (ez > 0 ? s_up : s_dn);
        const T* Cn = sm + slot * plane_stride + li + ey * PX + ex;
        T rest = T(0);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          T cn;
          if (i < NE) {
            cn = Cn[i * PXY];
            rest += cn;
          } else {
            cn = T(1) - rest;
          }
          const T d = cn - c[i];
          lap[i] += wk * d;
          if (ex != 0) gC[i][0] += (ex > 0) ? wk * d : -(wk * d);
          if (ey != 0) gC[i][1] += (ey > 0) ? wk * d : -(wk * d);
          if (ez != 0) gC[i][2] += (ez > 0) ? wk * d : -(wk * d);
        }
        const T dE = Cn[NE * PXY] - E0;
        if (ex != 0) gE[0] += (ex > 0) ? wk * dE : -(wk * dE);
        if (ey != 0) gE[1] += (ey > 0) ? wk * dE : -(wk * dE);
        if (ez != 0) gE[2] += (ez > 0) ? wk * dE : -(wk * dE);
      }
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      lap[i] *= T(6);
#pragma unroll
      for (int d = 0; d < 3; ++d) gC[i][d] *= T(3);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) gE[d] *= T(3);

    // ---- flux potential mu~ (factored; exact zero for an absent component)
    T mu[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T br = -(T(1) - T(3) * c[i] + T(2) * c[i] * c[i]);
#pragma unroll
      for (int l = 0; l < NC; ++l)
#pragma unroll
        for (int m = l + 1; m < NC; ++m)
          if (l != i && m != i) br += P.psi[i][l][m] * c[l] * c[m];
      T val = P.k34D * lap[i] + P.k12D * c[i] * br;
      if (a.flags & kFlagOmega) {
        T sx = T(0);
#pragma unroll
        for (int k2 = 0; k2 < NC; ++k2)
#pragma unroll
          for (int l = k2 + 1; l < NC; ++l)
            if (k2 != i && l != i) sx += P.xt[i][k2][l] * (c[k2] * c[k2]) * (c[l] * c[l]);
        T sy = T(0);
#pragma unroll
        for (int l = 0; l < NC; ++l) {
          if (l == i) continue;
          T inner = T(0);
#pragma unroll
          for (int m = 0; m < NC; ++m)
            if (m != i && m != l) inner += P.zt[i][l][m] * c[m];
          sy += c[l] * c[l] * inner;
        }
        val += P.k12D * P.omega_stab * c[i] * (sx + c[i] * sy);
      }
      mu[i] = val;
    }

    // ---- surface tension force + body force
    T F[3];
    if (a.flags & kFlagPotential) {
      F[0] = F[1] = F[2] = T(0);
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        T mraw = T(0);
#pragma unroll
        for (int k2 = 0; k2 < NC; ++k2)
          if (k2 != i)
            mraw += P.beta[i][k2] * (fprime(c[i]) - fprime(c[i] + c[k2])) + P.kappa[i][k2] * lap[k2];
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] += mraw * gC[i][d];
      }
    } else {
      F[0] = gE[0];
      F[1] = gE[1];
      F[2] = gE[2];
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        T kl = T(0);
#pragma unroll
        for (int j = 0; j < NC; ++j)
          if (j != i) kl += P.kappa[i][j] * lap[j];
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] += kl * gC[i][d];
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] += P.fb[d];

    // ---- hydrodynamic moments
    const size_t node = size_t(x) + size_t(a.nx) * (size_t(y) + size_t(a.ny) * size_t(z));
    const FS* fsrc = static_cast<const FS*>(a.f_src);
    T f[Q];
    f[0] = T(0);
#pragma unroll
    for (int k = 1; k < Q; ++k) f[k] = S::ld(fsrc, size_t(k - 1) * n + node);
    T v[3] = {T(0), T(0), T(0)};
    T fsum = T(0);
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      fsum += f[k];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (L::e[k][d] != 0) v[d] += (L::e[k][d] > 0) ? f[k] : -f[k];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] += T(0.5) * F[d];
    const T vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    T sk[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      T ev = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (L::e[k][d] != 0) ev += (L::e[k][d] > 0) ? v[d] : -v[d];
      sk[k] = static_cast<T>(L::w[k]) * (T(3) * ev + T(4.5) * ev * ev - T(1.5) * vv);
    }
    const T Pn = static_cast<T>((1.0 / 3.0) / (1.0 - L::w[0])) * (fsum + sk[0]);

    if constexpr (FIELDS) {
      double* out = a.fields;
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        out[size_t(P.uidx[i]) * n + node] = static_cast<double>(c[i]);
        out[size_t(NC + 7 + P.uidx[i]) * n + node] = (i < NE) ? static_cast<double>(mu[i]) : 0.0;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        out[size_t(NC + d) * n + node] = static_cast<double>(v[d]);
        out[size_t(NC + 4 + d) * n + node] = static_cast<double>(F[d]);
      }
      out[size_t(NC + 3) * n + node] = static_cast<double>(Pn);
      return;
    }

    // ---- node relaxation rates: majority component, lowest user index on ties
    T best = c[0];
    int bestu = P.uidx[0];
    T wp = P.omega_p[0], wm = P.omega_m[0];
#pragma unroll
    for (int i = 1; i < NC; ++i) {
      const int u = P.uidx[i];
      if (c[i] > best || (c[i] == best && u < bestu)) {
        best = c[i];
        bestu = u;
        wp = P.omega_p[i];
        wm = P.omega_m[i];
      }
    }

    // ---- streaming destinations (push), halfway bounce-back at walls
    int dst[Q];
    int dir[Q];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const int ex = L::e[k][0], ey = L::e[k][1], ez = L::e[k][2];
      int X = x + ex, Y = y + ey, Z = z + ez;
      bool wall = false;
      if (ex != 0) {
        if (X < 0 || X >= a.nx) {
          if (a.wall_x) wall = true;
          else X = (X < 0) ? X + a.nx : X - a.nx;
        }
      }
      if (ey != 0) {
        if (Y < 0 || Y >= a.ny) {
          if (a.wall_y) wall = true;
          else Y = (Y < 0) ? Y + a.ny : Y - a.ny;
        }
      }
      if (ez != 0) {
        if (Z < 0 || Z >= a.nz) {
          if (a.wall_z) wall = true;
          else Z = (Z < 0) ? Z + a.nz : Z - a.nz;
        }
      }
      const int kb = (k & 1) ? k + 1 : k - 1;
      if (wall) {
        dst[k] = static_cast<int>(node);
        dir[k] = kb;
      } else {
        dst[k] = X + a.nx * (Y + a.ny * Z);
        dir[k] = k;
      }
    }

    // ---- TRT collision of f with forcing
    FS* fdst = static_cast<FS*>(a.f_dst);
    const T vF = v[0] * F[0] + v[1] * F[1] + v[2] * F[2];
    const T cP = T(3) * Pn;
    const T hp = T(0.5) * (T(1) - T(0.5) * wp);
    const T hm = T(0.5) * (T(1) - T(0.5) * wm);
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
      const int kb = k + 1;
      const T wk = static_cast<T>(L::w[k]);
      T ev = T(0), eF = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (L::e[k][d] != 0) {
          ev += (L::e[k][d] > 0) ? v[d] : -v[d];
          eF += (L::e[k][d] > 0) ? F[d] : -F[d];
        }
      const T feq_k = wk * cP + sk[k];
      const T feq_b = wk * cP + sk[kb];
      const T Fk = wk * (T(3) * eF + T(9) * ev * eF - T(3) * vF);
      const T Fb = wk * (-T(3) * eF + T(9) * ev * eF - T(3) * vF);
      const T fp = T(0.5) * (f[k] + f[kb]), fm = T(0.5) * (f[k] - f[kb]);
      const T ep = T(0.5) * (feq_k + feq_b), em = T(0.5) * (feq_k - feq_b);
      const T sym = -wp * (fp - ep) + hp * (Fk + Fb);
      const T asym = -wm * (fm - em) + hm * (Fk - Fb);
      const T post_k = f[k] + sym + asym;
      const T post_b = f[kb] + sym - asym;
      fdst[size_t(dir[k] - 1) * n + size_t(dst[k])] = S::pack(post_k);
      fdst[size_t(dir[kb] - 1) * n + size_t(dst[kb])] = S::pack(post_b);
    }

    // ---- BGK collision of g towards the rest-form equilibrium
    FS* gkdst = static_cast<FS*>(a.gk_dst);
    G0S* g0dst = static_cast<G0S*>(a.g0_dst);
    const FS* gksrc = static_cast<const FS*>(a.gk_src);
    const G0S* g0src = static_cast<const G0S*>(a.g0_src);
    (void)g0src;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const T ci = c[i];
      const T mm = P.m * mu[i];
      T moved = T(0);
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        T post = ci * sk[k] - static_cast<T>(L::w[k]) * mm;
        if (a.flags & kFlagNeedG) {
          const T gv = S::ld(gksrc, (size_t(i) * (Q - 1) + (k - 1)) * n + node);
          post = gv - (gv - post) * P.inv_tau_g[i];
        }
        const FS q = S::pack(post);
        moved += S::unpack(q);
        gkdst[(size_t(i) * (Q - 1) + size_t(dir[k] - 1)) * n + size_t(dst[k])] = q;
      }
      g0dst[size_t(i) * n + node] = static_cast<G0S>(ci - moved);
    }
  };

  if constexpr (NPL == 3) {
    load_plane(0, z0 - 1);
    load_plane(1, z0);
    for (int z = z0; z < z1; ++z) {
      const int r = z - z0;
      const int s_dn = r % 3, s_c = (r + 1) % 3, s_up = (r + 2) % 3;
      load_plane(s_up, z + 1);
      __syncthreads();
      if (active) process(z, s_dn, s_c, s_up);
      __syncthreads();
    }
  } else {
    load_plane(0, 0);
    __syncthreads();
    if (active) process(0, 0, 0, 0);
  }
}

// ------------------------------------------------------------------ k_init
template <class L, int NC, int ST>
__global__ void __launch_bounds__(256) k_init(InitArgs a) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  constexpr int Q = L::Q;
  constexpr int NE = NC - 1;
  const DevParams<T>& P = *static_cast<const DevParams<T>*>(a.params);
  const size_t n = static_cast<size_t>(a.n);
  FS* f = static_cast<FS*>(a.f);
  FS* gk = static_cast<FS*>(a.gk);
  G0S* g0 = static_cast<G0S*>(a.g0);
  for (size_t node = blockIdx.x * size_t(256) + threadIdx.x; node < n;
       node += size_t(gridDim.x) * 256) {
    double v[3] = {0.0, 0.0, 0.0};
    double Pn = 0.0;
    if (a.v)
      for (int d = 0; d < 3; ++d) v[d] = a.v[size_t(d) * n + node];
    if (a.P) Pn = a.P[node];
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      double ev = 0.0;
      for (int d = 0; d < 3; ++d) ev += L::e[k][d] * v[d];
      const double s = L::w[k] * (3.0 * ev + 4.5 * ev * ev - 1.5 * vv);
      f[size_t(k - 1) * n + node] = S::pack(static_cast<T>(3.0 * L::w[k] * Pn + s));
    }
    for (int i = 0; i < NE; ++i) {
      g0[size_t(i) * n + node] = static_cast<G0S>(a.C[size_t(P.uidx[i]) * n + node]);
      for (int k = 1; k < Q; ++k) gk[(size_t(i) * (Q - 1) + (k - 1)) * n + node] = S::pack(T(0));
    }
  }
}

// ---------------------------------------------------------------- k_reduce
#if !defined(NFLBM_UNIT_STORE) || NFLBM_UNIT_STORE < 0
// Record per block: mass[N], mom[3], maxabs[N], minc[N], maxdev, cv[3], cmass, nan.
__host__ __device__ int reduce_record_len(int N) { return 3 * N + 9; }

__device__ __forceinline__ double shfl_down_d(double v, int off) { return __shfl_down(v, off, 64); }

template <int OP>  // 0 sum, 1 max, 2 min
__device__ double block_reduce(double v, double* scratch) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = shfl_down_d(v, off);
    if (OP == 0) v += o;
    else if (OP == 1) v = fmax(v, o);
    else v = fmin(v, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double r = scratch[0];
  for (int q = 1; q < 4; ++q) {
    if (OP == 0) r += scratch[q];
    else if (OP == 1) r = fmax(r, scratch[q]);
    else r = fmin(r, scratch[q]);
  }
  return r;
}

__global__ void __launch_bounds__(256) k_reduce_partial(ReduceArgs a) {
  __shared__ double scratch[4];
  const int N = a.N;
  const size_t n = static_cast<size_t>(a.n);
  const int rec = reduce_record_len(N);
  double* out = a.partial + size_t(blockIdx.x) * rec;
  const double* f = a.fields;
  const size_t per = (n + a.blocks - 1) / a.blocks;
  const size_t lo = size_t(blockIdx.x) * per;
  const size_t hi = lo + per < n ? lo + per : n;
  // one pass per quantity keeps the register footprint small
  for (int q = 0; q < rec; ++q) {
    int op = 0;
    double acc;
    if (q < N) { acc = 0.0; }
    else if (q < N + 3) { acc = 0.0; }
    else if (q < 2 * N + 3) { acc = 0.0; op = 1; }
    else if (q < 3 * N + 3) { acc = 1e300; op = 2; }
    else if (q == 3 * N + 3) { acc = 0.0; op = 1; }
    else { acc = 0.0; }
    for (size_t node = lo + threadIdx.x; node < hi; node += 256) {
      double val;
      if (q < N) val = f[size_t(q) * n + node];
      else if (q < N + 3) val = f[size_t(q) * n + node];
      else if (q < 2 * N + 3) val = fabs(f[size_t(q - N - 3) * n + node]);
      else if (q < 3 * N + 3) val = f[size_t(q - 2 * N - 3) * n + node];
      else if (q == 3 * N + 3) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) s += f[size_t(i) * n + node];
        val = fabs(s - 1.0);
      } else if (q < 3 * N + 7) {
        val = f[size_t(a.vcm_comp) * n + node] * f[size_t(N + q - 3 * N - 4) * n + node];
      } else if (q == 3 * N + 7) {
        val = f[size_t(a.vcm_comp) * n + node];
      } else {
        // NaN / Inf anywhere in the node's fields
        double s = 0.0;
        for (int r = 0; r < 2 * N + 7; ++r) s += f[size_t(r) * n + node] * 0.0;
        val = (s == 0.0) ? 0.0 : 1.0;
      }
      if (op == 0) acc += val;
      else if (op == 1) acc = fmax(acc, val);
      else acc = fmin(acc, val);
    }
    double r;
    if (op == 0) r = block_reduce<0>(acc, scratch);
    else if (op == 1) r = block_reduce<1>(acc, scratch);
    else r = block_reduce<2>(acc, scratch);
    if (threadIdx.x == 0) out[q] = r;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(64) k_reduce_final(ReduceArgs a) {
  const int N = a.N;
  const int rec = reduce_record_len(N);
  for (int q = threadIdx.x; q < rec; q += 64) {
    double acc = a.partial[q];
    for (int b = 1; b < a.blocks; ++b) {
      const double v = a.partial[size_t(b) * rec + q];
      if (q < N + 3) acc += v;
      else if (q < 2 * N + 3) acc = fmax(acc, v);
      else if (q < 3 * N + 3) acc = fmin(acc, v);
      else if (q == 3 * N + 3) acc = fmax(acc, v);
      else acc += v;
    }
    a.out[q] = acc;
  }
}
#endif

// --------------------------------------------------------------- dispatch
// kernels.hip is compiled once per storage precision (NFLBM_UNIT_STORE = 0, 1,
// 2), each unit instantiating the kernels of that precision, and once more
// (NFLBM_UNIT_STORE = -1) for the reductions and the precision switch.
template <int ST>
using TT = typename StoreT<ST>::T;

template <int ST>
size_t lds_bytes_for(int lat, int nc, int tx_log2) {
  const int TX = 1 << tx_log2, TY = 256 >> tx_log2;
  const size_t pxy = size_t(TX + 2) * (TY + 2);
  const int npl = lat == 1 ? 3 : 1;
  return npl * size_t(nc) * pxy * sizeof(TT<ST>);   // NE concentrations + E_B per slot
}

hipError_t update_st0(int lat, int nc, const StepArgs& a, bool fields, hipStream_t s);
hipError_t update_st1(int lat, int nc, const StepArgs& a, bool fields, hipStream_t s);
hipError_t update_st2(int lat, int nc, const StepArgs& a, bool fields, hipStream_t s);
hipError_t init_st0(int lat, int nc, const InitArgs& a, hipStream_t s);
hipError_t init_st1(int lat, int nc, const InitArgs& a, hipStream_t s);
hipError_t init_st2(int lat, int nc, const InitArgs& a, hipStream_t s);
hipError_t conc_st0(int lat, int nc, const StepArgs& a, hipStream_t s);
hipError_t conc_st1(int lat, int nc, const StepArgs& a, hipStream_t s);
hipError_t conc_st2(int lat, int nc, const StepArgs& a, hipStream_t s);

#if defined(NFLBM_UNIT_STORE) && NFLBM_UNIT_STORE >= 0

template <class L, int NC, int ST>
hipError_t launch_update_t(const StepArgs& a, bool fields, hipStream_t s) {
  const int blocks = a.tiles_x * a.tiles_y * a.chunks_z;
  const size_t lds = lds_bytes_for<ST>(L::DIM == 3 ? 1 : 0, NC, a.tx_log2);
  if (fields)
    hipLaunchKernelGGL((k_update<L, NC, ST, true>), dim3(blocks), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((k_update<L, NC, ST, false>), dim3(blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <class L, int NC, int ST>
hipError_t launch_init_t(const InitArgs& a, hipStream_t s) {
  long long blocks = (a.n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_init<L, NC, ST>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int Q, int ST>
hipError_t launch_conc_t(const StepArgs& a, int ne, hipStream_t s) {
  long long blocks = (a.n + 255) / 256;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL((k_conc<Q, ST>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a, ne);
  return hipGetLastError();
}

#define NFLBM_NC_SWITCH(NCV, CALL)        \
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

template <class L, int ST>
hipError_t update_nc(int nc, const StepArgs& a, bool fields, hipStream_t s) {
#define CALL_U(K) launch_update_t<L, K, ST>(a, fields, s)
  NFLBM_NC_SWITCH(nc, CALL_U)
#undef CALL_U
}

template <class L, int ST>
hipError_t init_nc(int nc, const InitArgs& a, hipStream_t s) {
#define CALL_I(K) launch_init_t<L, K, ST>(a, s)
  NFLBM_NC_SWITCH(nc, CALL_I)
#undef CALL_I
}

#define NFLBM_CAT2(a, b) a##b
#define NFLBM_CAT(a, b) NFLBM_CAT2(a, b)
#define NFLBM_ST NFLBM_UNIT_STORE

hipError_t NFLBM_CAT(update_st, NFLBM_ST)(int lat, int nc, const StepArgs& a, bool fields, hipStream_t s) {
  return lat == 0 ? update_nc<D2Q9, NFLBM_ST>(nc, a, fields, s) : update_nc<D3Q19, NFLBM_ST>(nc, a, fields, s);
}
hipError_t NFLBM_CAT(init_st, NFLBM_ST)(int lat, int nc, const InitArgs& a, hipStream_t s) {
  return lat == 0 ? init_nc<D2Q9, NFLBM_ST>(nc, a, s) : init_nc<D3Q19, NFLBM_ST>(nc, a, s);
}
hipError_t NFLBM_CAT(conc_st, NFLBM_ST)(int lat, int nc, const StepArgs& a, hipStream_t s) {
  return lat == 0 ? launch_conc_t<9, NFLBM_ST>(a, nc - 1, s) : launch_conc_t<19, NFLBM_ST>(a, nc - 1, s);
}

#else  // common unit

size_t update_lds_bytes(int lat, int nc, int store, int tx_log2) {
  switch (store) {
    case kStoreF64: return lds_bytes_for<kStoreF64>(lat, nc, tx_log2);
    case kStoreF32: return lds_bytes_for<kStoreF32>(lat, nc, tx_log2);
    default: return lds_bytes_for<kStoreF16S>(lat, nc, tx_log2);
  }
}

hipError_t launch_update(int lat, int nc, int store, const StepArgs& a, bool fields, hipStream_t s) {
  switch (store) {
    case kStoreF64: return update_st0(lat, nc, a, fields, s);
    case kStoreF32: return update_st1(lat, nc, a, fields, s);
    case kStoreF16S: return update_st2(lat, nc, a, fields, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_init(int lat, int nc, int store, const InitArgs& a, hipStream_t s) {
  switch (store) {
    case kStoreF64: return init_st0(lat, nc, a, s);
    case kStoreF32: return init_st1(lat, nc, a, s);
    case kStoreF16S: return init_st2(lat, nc, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_conc(int lat, int nc, int store, const StepArgs& a, hipStream_t s) {
  switch (store) {
    case kStoreF64: return conc_st0(lat, nc, a, s);
    case kStoreF32: return conc_st1(lat, nc, a, s);
    case kStoreF16S: return conc_st2(lat, nc, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(a.blocks), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

#endif

}  // namespace nflbm
