// Device code of the N-component free-energy LBM time step for gfx950.
//
// Storage (pull streaming): each population set holds the POST-COLLISION
// populations of the previous step; a node gathers its post-streaming values
// f_k(x) = f*_k(x - e_k), or f*_kbar(x) when x - e_k lies inside a wall
// (halfway bounce-back).  Every store of the update is then aligned with the
// node that computes it, and only loads are shifted.
//
// Layout, node = x + nx (y + ny z), direction arrays fstride / gstride apart:
//   f [k-1][node]            moving hydrodynamic populations, k = 1..Q-1
//   gk[k-1][node][i]         moving populations of the evolved components,
//                            component innermost: one vector access moves
//                            all components of a direction
//   g0[node][i]              rest populations of the evolved components
//   conc[node][i]            reconstructed concentrations (compute precision)
//   eb[node]                 bulk free energy E_B of the reconstructed C
//
// One time step = two launches:
//   k_conc    C_i = sum_k g_{i,k} of the evolved components (zeroth moment of
//             g, Sec. III B), gathering the streamed populations, and E_B(C).
//   k_update  per node: C of all components and E_B from an LDS halo tile
//             (the implicit C as 1 - sum of the others), the isotropic
//             gradient/Laplacian stencils (Eq. gradstencil) with the wall
//             rule, the flux potential mu~ in factored form, the conservative
//             surface-tension force (Eq. Fsnew), v and P (Eqs. nmom, pres),
//             node viscosity, TRT collision with forcing (Eqs. TRT, FTRT,
//             hydroforce) and BGK collision of g (Eq. glbe).
// The concentration equilibrium is the rest-population form
//   g^eq_{i,0} = C_i (1 + s_0) + (1 - w_0) m mu~_i,  g^eq_{i,k} = C_i s_k - w_k m mu~_i;
// the rest population is written as C_i minus the stored moving populations,
// which equals g^eq_{i,0} in exact arithmetic and keeps node mass to the
// rounding of one value in every storage precision.
//
// Workgroups are 256 threads covering a TX x TY tile of the x-y plane.  The
// D2Q9 update loads one LDS plane; the D3Q19 update marches along z through
// zchunk planes with a rolling window of LDS planes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device.h"

namespace nflbm {

// ------------------------------------------------------------------ k_conc
// One node per thread over TX x TY tiles of one z plane: C of the evolved
// components from the gathered g, and the bulk free energy E_B(C), which the
// update reads for its gradient.  b is the workgroup's tile index within the
// simulation (x fastest, then y, then z).
template <class L, int NE, int ST, bool WALLS>
__device__ __forceinline__ void conc_tile(const StepArgs& a,
                                          const DevParams<typename StoreT<ST>::T>* __restrict__ Pp, int b) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  constexpr int Q = L::Q;
  constexpr int NC = NE + 1;
  const DevParams<T>& P = *gptr<const DevParams<T>>(Pp);
  const int TX = 1 << a.tx_log2;
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x >> a.tx_log2;
  const int tile_x = a.tile_x0 + (b % a.tiles_x) * a.tile_xstep;
  b /= a.tiles_x;
  const int tile_y = b % a.tiles_y;
  const int z = b / a.tiles_y;
  const int x = tile_x * TX + tx, y = tile_y * (256 >> a.tx_log2) + ty;
  if (x >= a.nx || y >= a.ny) return;
  const uint32_t node = uint32_t(x) + uint32_t(a.nx) * (uint32_t(y) + uint32_t(a.ny) * uint32_t(z));
  const Nbr nb = neighbours<L, WALLS>(x, y, z, a);
  if (solid_node<WALLS>(nb)) {
    T zero[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) zero[e] = T(0);
    vst<T, NE>(at(gptr<T>(a.conc), node * NE), zero);
    *at(gptr<T>(a.eb), node) = T(0);
    return;
  }
  const G0S* g0 = gptr<const G0S>(a.g0_src);
  const FS* gk = gptr<const FS>(a.gk_src);
  // The small moving populations are summed first and the O(1) rest
  // population added last: one rounding at the scale of C per node.  Adding
  // them one by one onto the rest population would round every addition at
  // that scale, with errors that are alike at neighbouring nodes of a smooth
  // field and accumulate into a drift of the total mass in float storage.
  T s[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) s[e] = T(0);
  // convective outflow: the boundary plane's post-streaming populations (all
  // k) are held in the plane buffer, not pulled
  const int op = (WALLS && a.out_face >= 0) ? outflow_plane_index(a.out_face, 0, x, y, z, a) : -1;
  if (WALLS && op >= 0) {
    const uint32_t PL = outflow_plane_size(a.out_face, a.nx, a.ny, a.nz);
    const T* og = gptr<const T>(a.out_g);
    for (int e = 0; e < NE; ++e) {
      T m = T(0);
      for (int k = 1; k < Q; ++k) m += og[(uint32_t(e) * Q + k) * PL + op];
      s[e] = og[uint32_t(e) * Q * PL + op] + m;
    }
  } else {
    // open faces: a population entering across one is minus this node's own
    // opposite one plus g^eq_k + g^eq_kbar of the face (anti-bounce-back)
    const FaceBC<T>* FB = gptr<const FaceBC<T>>(a.faces);
    const int open = (WALLS && FB) ? FB->open : 0;
    const size_t gst = static_cast<size_t>(a.gstride);
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      FS v[NE];
      if (pulled_from_wall<L, WALLS>(nb, k))
        vld_nt<FS, NE>(at(gk + size_t(opposite(k) - 1) * gst, node * NE), v);
      else
        vld_nt<FS, NE>(at(gk + size_t(k - 1) * gst, upstream<L>(nb, k) * NE), v);
      const int fc = entry_face<L, WALLS>(nb, k, open);
      if (fc >= 0) {
#pragma unroll
        for (int e = 0; e < NE; ++e) s[e] += FB->gsum[fc][e][k] - S::unpack(v[e]);
      } else {
#pragma unroll
        for (int e = 0; e < NE; ++e) s[e] += S::unpack(v[e]);
      }
    }
    {
      G0S r[NE];
      vld_nt<G0S, NE>(at(g0, node * NE), r);
#pragma unroll
      for (int e = 0; e < NE; ++e) s[e] = static_cast<T>(r[e]) + s[e];
    }
  }
  vst<T, NE>(at(gptr<T>(a.conc), node * NE), s);
  T c[NC];
  T rest = T(0);
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    c[e] = s[e];
    rest += s[e];
  }
  c[NE] = T(1) - rest;
  *at(gptr<T>(a.eb), node) = bulk_energy<NC, T>(c, P);
}

template <class L, int NE, int ST, bool WALLS>
__global__ void __launch_bounds__(256)
k_conc(StepArgs a, const DevParams<typename StoreT<ST>::T>* __restrict__ Pp) {
  conc_tile<L, NE, ST, WALLS>(a, Pp, static_cast<int>(blockIdx.x));
}

// Batch form: workgroup w works on tile work[w].y of simulation m = work[w].x,
// whose arguments are args[m] and coefficient tables params[m].
template <class L, int NE, int ST, bool WALLS>
__global__ void __launch_bounds__(256)
k_conc_batch(const StepArgs* __restrict__ args, const DevParams<typename StoreT<ST>::T>* __restrict__ params,
             const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const StepArgs a = args[w.x];
  conc_tile<L, NE, ST, WALLS>(a, params + w.x, w.y);
}

// --------------------------------------------------- k_conc, moment form
// With tau_g = 1 the post-collision populations of every evolved component
// are its equilibria, C_i s_k(v) - w_k m mu~_i (Eq. glbe with tau_g = 1,
// Eq. geq), so the state holds, per node, the C_i the collision used, mu~_i,
// v and v.v instead of the 19 (N - 1) populations.  This kernel re-forms them
// where they are needed:
//   C_i(x, t+1) = g^eq_{i,0}(x) + sum_{k>=1} g*_{i,k}(x - e_k)
// (rest population of Eq. geq plus the streamed moving populations, halfway
// bounce-back at walls), in the compute precision.  The incoming sum is
// grouped as sum_k C s_k - m sum_k w_k mu~, and the rest population is formed
// directly rather than as C minus the node's own outgoing populations: the
// two forms of g then agree to rounding instead of bit for bit, for a third
// of this kernel's arithmetic.  Mass is kept to the rounding of C at each
// node (no systematic drift; see the comment at the final sum).  The per-node
// records of the tile and a one-node halo sit in LDS one plane at a time: in
// D3Q19 a workgroup marches along z and each plane's records are added to
// the three nodes of every column that they reach (the planes below, at and
// above it), so that only one plane of records occupies LDS and more
// workgroups share a CU.
// LDS record of one position: C in [0, NEP), mu~ in [NEP, 2 NEP), then v and
// v.v, and in the record form of f the four values (fB, F), with NEP = NE
// rounded up to 4 so every group starts 16-byte aligned and moves with
// vector reads.  The record is padded to an odd multiple of 16
// bytes (12 or 20 floats, 14 or 22 doubles): consecutive positions then start
// in different 16-byte bank groups, so a wavefront's reads of a row of
// positions do not collide on banks.
// In FP64 the fields are stored field-major instead (field f of position p at
// f * PXY + p, NEP = NE, no padding): its 8-byte reads of consecutive
// positions are conflict-free, and the FP64 reconstruction measured faster
// that way, while FP32 and FP16S measured faster with records.
template <class T>
constexpr bool moment_aos() { return sizeof(T) == 4; }
template <int NE, class T>
constexpr int moment_nep() { return moment_aos<T>() ? (NE + 3) / 4 * 4 : NE; }
template <int NE, class T, bool FR>
constexpr int moment_record() {
  const int r = 2 * moment_nep<NE, T>() + 4 + (FR ? 4 : 0);
  if (!moment_aos<T>()) return r;
  return (r * int(sizeof(T)) / 16) % 2 == 1 ? r : r + 16 / int(sizeof(T));
}

template <class L, int NE, int ST, bool WALLS, int TXL, bool FR>
__device__ __forceinline__ void conc_tile_m(const StepArgs& a,
                                            const DevParams<typename StoreT<ST>::T>* __restrict__ Pp, int b,
                                            unsigned char* smem_raw) {
  using S = StoreT<ST>;
  using T = typename S::T;
  constexpr int Q = L::Q;
  constexpr int NC = NE + 1;
  constexpr bool D3 = (L::DIM == 3);
  constexpr bool AOS = moment_aos<T>();
  constexpr int NEP = moment_nep<NE, T>();
  constexpr int REC = moment_record<NE, T, FR>();
  constexpr int NF = 2 * NE + 4;          // field-major: first field of (fB, F)
  constexpr int TX = 1 << TXL;
  constexpr int TY = 256 >> TXL;
  constexpr int PX = TX + 2;
  constexpr int PXY = PX * (TY + 2);
  T* sm = reinterpret_cast<T*>(smem_raw);
  const DevParams<T>* P0 = gptr<const DevParams<T>>(Pp);
  const int tid = threadIdx.x;
  const int tx = tid & (TX - 1);
  const int ty = tid >> TXL;
  const int tile_x = a.tile_x0 + (b % a.tiles_x) * a.tile_xstep;
  b /= a.tiles_x;
  const int tile_y = b % a.tiles_y;
  const int chunk = b / a.tiles_y;
  const int x0 = tile_x * TX, y0 = tile_y * TY;
  const int z0 = chunk * a.zchunk;
  const int z1 = min(z0 + a.zchunk, a.nz);
  const int x = x0 + tx, y = y0 + ty;
  const bool active = (x < a.nx) && (y < a.ny);
  const uint32_t nx = a.nx, nxy = uint32_t(a.nx) * uint32_t(a.ny);
  const T* cprev = gptr<const T>(a.cprev);
  // first step after set_fields: a node's f is its own record's equilibrium
  const bool flocal = FR && (a.flags & kFlagFLocal);

  uint32_t fill_off[2];
  bool fill_ok[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int idx = tid + 256 * r;
    fill_ok[r] = idx < PXY;
    fill_off[r] = 0;
    if (fill_ok[r]) {
      const int ly = idx / PX;
      const int lx = idx - ly * PX;
      int gx = x0 + lx - 1, gy = y0 + ly - 1;
      if (gx < 0 || gx >= a.nx) {
        if (WALLS && a.wall_x) fill_ok[r] = false;
        else gx = wrap(gx, a.nx);
      }
      if (gy < 0 || gy >= a.ny) {
        if (WALLS && a.wall_y) fill_ok[r] = false;
        else gy = wrap(gy, a.ny);
      }
      fill_off[r] = uint32_t(gx) + nx * uint32_t(gy);
    }
  }

  // Records of plane gz into the LDS plane, one record per position; false
  // for a plane beyond a wall face (nothing is loaded).  Positions inside a
  // wall stay unfilled: a population pulled from a wall is this node's own,
  // so they are never read.
  auto load_plane = [&](int gz) -> bool {
    T* base = sm;
    if (gz < 0 || gz >= a.nz) {
      if (WALLS && a.wall_z) return false;
      gz = (gz < 0) ? gz + a.nz : gz - a.nz;
    }
    const uint32_t zoff = uint32_t(gz) * nxy;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!fill_ok[r]) continue;
      const int idx = tid + 256 * r;
      const uint32_t node = fill_off[r] + zoff;
      T cc[NEP], mm[NEP], vv[4], ff[4];
#pragma unroll
      for (int e = NE; e < NEP; ++e) cc[e] = mm[e] = T(0);
      vld<T, NE>(at(cprev, node * NE), reinterpret_cast<T(&)[NE]>(cc));
      rec_load<S, NE>(a.mu, node * NE, reinterpret_cast<T(&)[NE]>(mm), T(S::mu_scale));
      rec_load<S, 4>(a.vel, node * 4, vv, T(S::vel_scale));
      if constexpr (FR) rec_load<S, 4>(a.frec, node * 4, ff, T(S::vel_scale));
      if constexpr (AOS) {
        T* rec = base + idx * REC;
        vst<T, NEP>(rec, cc);
        vst<T, NEP>(rec + NEP, mm);
        vst<T, 4>(rec + 2 * NEP, vv);
        if constexpr (FR) vst<T, 4>(rec + 2 * NEP + 4, ff);
      } else {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          base[e * PXY + idx] = cc[e];
          base[(NE + e) * PXY + idx] = mm[e];
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) base[(2 * NE + d) * PXY + idx] = vv[d];
        if constexpr (FR) {
#pragma unroll
          for (int d = 0; d < 4; ++d) base[(NF + d) * PXY + idx] = ff[d];
        }
      }
    }
    return true;
  };
  // C, mu~ and (v, -3/2 v.v) of the position at rec (a record start, or in the
  // field-major layout the position's slot in the first field)
  auto read_pos = [&](const T* rec, T (&cs)[NEP], T (&ms)[NEP], T (&v4)[4]) {
    if constexpr (AOS) {
      vld<T, NEP>(rec, cs);
      vld<T, NEP>(rec + NEP, ms);
      vld<T, 4>(rec + 2 * NEP, v4);
    } else {
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        cs[e] = rec[e * PXY];
        ms[e] = rec[(NE + e) * PXY];
      }
#pragma unroll
      for (int d = 0; d < 4; ++d) v4[d] = rec[(2 * NE + d) * PXY];
    }
  };
  constexpr int PSTEP = AOS ? REC : 1;   // distance between positions
  // v and (fB, F) of the position at rec (record form of f)
  auto read_f = [&](const T* rec, T (&v3)[3], T (&f4)[4]) {
    if constexpr (AOS) {
      T v4[4];
      vld<T, 4>(rec + 2 * NEP, v4);
      vld<T, 4>(rec + 2 * NEP + 4, f4);
      v3[0] = v4[0]; v3[1] = v4[1]; v3[2] = v4[2];
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) v3[d] = rec[(2 * NE + d) * PXY];
#pragma unroll
      for (int d = 0; d < 4; ++d) f4[d] = rec[(NF + d) * PXY];
    }
  };

  // Per-target sums of the z march.  s holds the target's net change of C
  // from its incoming populations, sum_k (C s_k - w_k m mu~) of their
  // sources, with the rest-population term C s_0 + (1 - w_0) m mu~ of its own
  // record folded in; c is the node's own C.  With float records and f as
  // populations (CLASS), s and sd instead hold sum (C s_k / w_k - m mu~) over
  // the axis and the diagonal directions, weighted once at the end, and d0
  // the rest-population term: the per-direction weight is then not applied.
  // Record form of f: fm sums the incoming f (sum_k f_k), jm their e_k f_k.
  constexpr bool CLASS = AOS && !FR;
  struct Acc {
    T s[NE], sd[NE], c[NE], d0[NE];
    T fm, jm[3];
    bool solid;
  };
  auto zero_acc = [&](Acc& A) {
#pragma unroll
    for (int e = 0; e < NE; ++e) A.s[e] = A.sd[e] = A.c[e] = A.d0[e] = T(0);
    A.fm = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) A.jm[d] = T(0);
    A.solid = false;
  };
  auto add_f_value = [&](Acc& A, T fk, int kin) {
    A.fm += fk;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (L::e[kin][d] != 0) A.jm[d] += (L::e[kin][d] > 0) ? fk : -fk;
  };

  // A source position's record as read from LDS (f4 only with the record
  // form of f)
  struct Rec {
    T cs[NEP], ms[NEP], v4[4], f4[4];
  };
  // WF (std::true_type / std::false_type): whether the f* of the sources are
  // gathered (false only on the first step after set_fields)
  auto read_rec = [&](const T* src, Rec& R, auto WF) {
    read_pos(src, R.cs, R.ms, R.v4);
    if constexpr (FR && decltype(WF)::value) {
      if constexpr (AOS) {
        vld<T, 4>(src + 2 * NEP + 4, R.f4);
      } else {
#pragma unroll
        for (int d = 0; d < 4; ++d) R.f4[d] = src[(NF + d) * PXY];
      }
    }
  };
  // One incoming population of direction kd from the source record R:
  // s_k / w_k = (e.v)(4.5 e.v +- 3) - 3/2 v.v (Eqs. feq, geq) from the
  // source's v, formed through the odd member of the pair; negm = -m.
  // With the record form of f (and with_f), the same source's f*_kd is added
  // to the moments of the f arriving along e_kin (kin = kd, or its opposite
  // where the population is bounced back), from the same s_k.
  // NEG (std::true_type): the population of g enters with the opposite sign
  // (anti-bounce-back at an open face); f keeps its sign.
  auto acc_rec = [&](Acc& A, const Rec& R, int kd, int kin, auto WF, T negm, auto NEG) {
    constexpr bool N_ = decltype(NEG)::value;
    const int kp = (kd & 1) ? kd : kd - 1;
    const T vs[3] = {R.v4[0], R.v4[1], R.v4[2]};
    const T ev = proj<L>(kp, vs);
    const T u = fma(ev, fma(T(4.5), ev, (kd & 1) ? T(3) : -T(3)), R.v4[3]);
    const T wk = static_cast<T>(L::w[kp]);
    const T gm = N_ ? -negm : negm;
    if constexpr (CLASS) {
      if (L::w[kp] == L::w[1]) {
#pragma unroll
        for (int e = 0; e < NE; ++e) A.s[e] = fma(N_ ? -R.cs[e] : R.cs[e], u, fma(gm, R.ms[e], A.s[e]));
      } else {
#pragma unroll
        for (int e = 0; e < NE; ++e) A.sd[e] = fma(N_ ? -R.cs[e] : R.cs[e], u, fma(gm, R.ms[e], A.sd[e]));
      }
    } else {
      const T wu = wk * u;
      const T mw = gm * wk;
#pragma unroll
      for (int e = 0; e < NE; ++e) A.s[e] = fma(N_ ? -R.cs[e] : R.cs[e], wu, fma(mw, R.ms[e], A.s[e]));
      if constexpr (FR && decltype(WF)::value) {
        // f*_k = w_k s_k / w_k + w_k [fB + (e.F)(9/2 e.v +- 3/2)]
        const T F[3] = {R.f4[1], R.f4[2], R.f4[3]};
        const T eF = proj<L>(kp, F);
        const T t = fma(eF, fma(T(4.5), ev, (kd & 1) ? T(1.5) : -T(1.5)), R.f4[0]);
        add_f_value(A, fma(wk, t, wu), kin);
      }
    }
  };
  auto add_source = [&](Acc& A, const T* src, int kd, int kin, auto WF, T negm) {
    Rec R;
    read_rec(src, R, WF);
    acc_rec(A, R, kd, kin, WF, negm, std::false_type{});
  };
  // open faces (anti-bounce-back for g, velocity Dirichlet for f): the
  // population entering along e_k across face fc is minus (f: plus) this
  // node's own opposite one, plus g^eq_k + g^eq_kbar of the face (f: plus
  // 2 w_k (e_k . v_b) / c_s^2).  On the first step after set_fields the
  // incoming populations are the initial ones, g_k = 0 (and f from the
  // node's own record, added separately).
  const FaceBC<T>* FB = gptr<const FaceBC<T>>(a.faces);
  const int open = (WALLS && FB) ? FB->open : 0;
  const bool first = (a.flags & kFlagFLocal) != 0;
  auto add_open = [&](Acc& A, const T* own, int k, int fc, auto WF, T negm) {
    if (first) return;
    Rec R;
    read_rec(own, R, WF);
    acc_rec(A, R, opposite(k), k, WF, negm, std::true_type{});
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      if constexpr (CLASS) A.d0[e] += FB->gsum[fc][e][k];
      else A.s[e] += FB->gsum[fc][e][k];
    }
    if constexpr (FR && decltype(WF)::value) add_f_value(A, FB->fcorr[fc][k], k);
  };
  const int li = (ty + 1) * PX + (tx + 1);
  // record of the position x - e (in-plane part of e) in the LDS plane
  const T* corner = sm + (li - PX - 1) * PSTEP;
  auto src_at = [&](int ex, int ey) { return corner + ((1 - ey) * PX + (1 - ex)) * PSTEP; };

  // The populations held in plane p reach three targets of this column: the
  // node of plane p + 1 (directions with e_z = +1), the node of plane p
  // itself (in-plane directions, its rest population, and every population
  // bounced back at a wall, which is its own), and the node of plane p - 1
  // (e_z = -1).  A target is complete once plane t + 1 has been seen.
  auto plane_step = [&](int p, bool have, Acc& lo, Acc& mid, Acc& hi, auto WF) {
    const NFLBM_CONST DevParams<T>& P = *fresh_const(P0);
    const T negm = -P.m;
    const bool need_hi = D3 && have && p + 1 >= z0 && p + 1 < z1;
    const bool need_lo = D3 && have && p - 1 >= z0 && p - 1 < z1;
    // Away from walls, the node of plane p + 1 (directions (ex, ey, +1)) and
    // the node of plane p - 1 (directions (ex, ey, -1)) pull from the same
    // five positions of plane p: each record is read once for both.
    const bool merged = D3 && !WALLS && need_hi && need_lo;
    if (merged) {
#pragma unroll
      for (int k = 1; k < Q; ++k)
        if (L::e[k][2] == 1) {
          const int km = direction_of<L>(L::e[k][0], L::e[k][1], -1);
          Rec R;
          read_rec(src_at(L::e[k][0], L::e[k][1]), R, WF);
          acc_rec(hi, R, k, k, WF, negm, std::false_type{});
          acc_rec(lo, R, km, km, WF, negm, std::false_type{});
        }
    }
    if (!merged && need_hi) {
      const Nbr nb = neighbours<L, WALLS>(x, y, p + 1, a);
#pragma unroll
      for (int k = 1; k < Q; ++k)
        if (L::e[k][2] == 1 && !pulled_from_wall<L, WALLS>(nb, k))
          add_source(hi, src_at(L::e[k][0], L::e[k][1]), k, k, WF, negm);
    }
    if (p >= z0 && p < z1) {
      const Nbr nb = neighbours<L, WALLS>(x, y, p, a);
      mid.solid = solid_node<WALLS>(nb);
      const T* own = src_at(0, 0);
      {
        T cs[NEP], ms[NEP], v4[4];
        read_pos(own, cs, ms, v4);
        const T s0 = static_cast<T>(L::w[0]) * v4[3];
        const T m0 = moving_weight_sum<L, T>() * P.m;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          mid.c[e] = cs[e];
          const T d0 = fma(cs[e], s0, m0 * ms[e]);
          if constexpr (CLASS) mid.d0[e] = d0;
          else mid.s[e] += d0;
        }
      }
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        if (pulled_from_wall<L, WALLS>(nb, k)) {
          const int fc = entry_face<L, WALLS>(nb, k, open);
          if (WALLS && fc >= 0) add_open(mid, own, k, fc, WF, negm);
          else add_source(mid, own, opposite(k), k, WF, negm);
        } else if (L::e[k][2] == 0) {
          add_source(mid, src_at(L::e[k][0], L::e[k][1]), k, k, WF, negm);
        }
      }
      if constexpr (FR && !decltype(WF)::value) {
        // first step after set_fields: every f of the node is the
        // equilibrium of its own record (A0, v0)
        T f4[4], v3[3];
        read_f(own, v3, f4);
#pragma unroll
        for (int k = 1; k < Q; ++k) add_f_value(mid, static_cast<T>(L::w[k]) * f_scaled_local<L>(k, f4), k);
      }
    }
    if (!merged && need_lo) {
      // in the merged path's order (by the (ex, ey, +1) directions), so that
      // a node's sums do not depend on where the z runs start and end
      const Nbr nb = neighbours<L, WALLS>(x, y, p - 1, a);
#pragma unroll
      for (int k = 1; k < Q; ++k)
        if (L::e[k][2] == 1) {
          const int km = direction_of<L>(L::e[k][0], L::e[k][1], -1);
          if (!pulled_from_wall<L, WALLS>(nb, km)) add_source(lo, src_at(L::e[k][0], L::e[k][1]), km, km, WF, negm);
        }
    }
  };

  // C of a complete target: its own C plus the net change (rest population
  // less C, plus the streamed-in ones), the small terms summed first so that
  // they meet C in one rounding.  Added to C on its own, C s_0 (never
  // positive) would be lost below half an ulp at every node and step alike: a
  // steady mass gain in float storage (1e-5 per step on the 64^2 lens).
  auto finish = [&](const Acc& A, int z) {
    const uint32_t node = uint32_t(x) + nx * uint32_t(y) + nxy * uint32_t(z);
    T sum[NE];
    // convective outflow: the boundary plane's post-streaming populations
    // (every k) are the plane buffers, from which the outflow kernel that
    // wrote them (after the previous step, or when the state or the outflow
    // was set) has already formed this node's C, E_B and f moments
    if (WALLS && !A.solid && a.out_face >= 0 && outflow_plane_index(a.out_face, 0, x, y, z, a) >= 0) return;
    if (A.solid) {
#pragma unroll
      for (int e = 0; e < NE; ++e) sum[e] = T(0);
      vst<T, NE>(at(gptr<T>(a.conc), node * NE), sum);
      *at(gptr<T>(a.eb), node) = T(0);
      if constexpr (FR) {
        const T z4[4] = {T(0), T(0), T(0), T(0)};
        rec_store<S, 4, false>(a.fmom, node * 4, z4, T(S::vel_scale));
      }
      return;
    }
    if constexpr (FR) {
      // moments of the streamed f: sum_k f_k and sum_k e_k f_k
      const T fm[4] = {A.fm, A.jm[0], A.jm[1], A.jm[2]};
      rec_store<S, 4, true>(a.fmom, node * 4, fm, T(S::vel_scale));
    }
    const NFLBM_CONST DevParams<T>& P = *fresh_const(P0);
    T cn[NC];
    T rest = T(0);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      T d = A.s[e];
      if constexpr (CLASS) d = A.d0[e] + fma(static_cast<T>(L::w[1]), A.s[e], static_cast<T>(L::w[Q - 1]) * A.sd[e]);
      sum[e] = A.c[e] + d;
      cn[e] = sum[e];
      rest += sum[e];
    }
    cn[NE] = T(1) - rest;
    vst<T, NE>(at(gptr<T>(a.conc), node * NE), sum);
    *at(gptr<T>(a.eb), node) = bulk_energy<NC, T>(cn, P);
  };

  // One LDS plane: planes z0 - 1 .. z1 pass through it in turn (D2Q9: the
  // single plane), each read by three targets as above.
  auto march = [&](auto WF) {
    Acc lo, mid, hi;
    zero_acc(lo);
    zero_acc(mid);
    zero_acc(hi);
    const int p_first = D3 ? z0 - 1 : 0, p_last = D3 ? z1 : 0;
    for (int p = p_first; p <= p_last; ++p) {
      if (p != p_first) __syncthreads();      // every read of the previous plane is done
      const bool have = load_plane(p);
      __syncthreads();
      if (active) {
        plane_step(p, have, lo, mid, hi, WF);
        if (!D3) finish(mid, 0);
        else if (p - 1 >= z0) finish(lo, p - 1);
      }
      lo = mid;
      mid = hi;
      zero_acc(hi);
    }
  };
  if (flocal) march(std::false_type{});
  else march(std::true_type{});
}

template <class L, int NE, int ST, bool WALLS, int TXL, bool FR>
__global__ void __launch_bounds__(256)
k_conc_m(StepArgs a, const DevParams<typename StoreT<ST>::T>* __restrict__ Pp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nblocks = a.tiles_x * a.tiles_y * a.chunks_z;
  conc_tile_m<L, NE, ST, WALLS, TXL, FR>(a, Pp, xcd_remap(static_cast<int>(blockIdx.x), nblocks), smem_raw);
}

template <class L, int NE, int ST, bool WALLS, int TXL, bool FR>
__global__ void __launch_bounds__(256)
k_conc_m_batch(const StepArgs* __restrict__ args, const DevParams<typename StoreT<ST>::T>* __restrict__ params,
               const int2* __restrict__ work, int nblocks) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 w = work[xcd_remap(static_cast<int>(blockIdx.x), nblocks)];
  const StepArgs a = args[w.x];
  conc_tile_m<L, NE, ST, WALLS, TXL, FR>(a, params + w.x, w.y, smem_raw);
}

// Post-collision populations of the moment form written out in the
// population layout (g0 [node][i], gk [k-1][node][i] of the population form),
// for read-back; one node per thread.  With FP16S the moving ones are
// rounded to binary16 there, as that layout stores them.
template <class L, int NE, int ST>
__global__ void __launch_bounds__(256) k_expand_g(StepArgs a, const DevParams<typename StoreT<ST>::T>* __restrict__ Pp) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  constexpr int Q = L::Q;
  const size_t n = static_cast<size_t>(a.n);
  const size_t node = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (node >= n) return;
  const DevParams<T>& P = *gptr<const DevParams<T>>(Pp);
  T c[NE], mu[NE], vel[4];
  vld<T, NE>(gptr<const T>(a.cprev) + node * NE, c);
  rec_load<S, NE>(a.mu, uint32_t(node * NE), mu, T(S::mu_scale));
  rec_load<S, 4>(a.vel, uint32_t(node * 4), vel, T(S::vel_scale));
  const T v[3] = {vel[0], vel[1], vel[2]};
  const T base_s = vel[3];
  FS* gk = gptr<FS>(a.gk_dst);
#pragma unroll
  for (int k = 1; k < Q; k += 2) {
    const T ev = proj<L>(k, v);
    const T quad = quad_term<L>(ev, base_s);
    const T sk = s_pair_member<L>(k, ev, quad);
    const T sb = s_pair_member<L>(k + 1, ev, quad);
    const T mw = static_cast<T>(L::w[k]) * P.m;
    FS qk[NE], qb[NE];
    for (int e = 0; e < NE; ++e) {
      const T mmu = mw * mu[e];
      const T gk = g_post(c[e], sk, mmu), gb = g_post(c[e], sb, mmu);
      qk[e] = S::pack(gk);   // read-back layout of the population form
      qb[e] = S::pack(gb);
    }
    vst<FS, NE>(gk + size_t(k - 1) * size_t(a.gstride) + node * NE, qk);
    vst<FS, NE>(gk + size_t(k) * size_t(a.gstride) + node * NE, qb);
  }
  // the rest population as the reconstruction uses it (Eq. geq)
  const T s0 = static_cast<T>(L::w[0]) * base_s;
  const T m0 = moving_weight_sum<L, T>() * P.m;
  G0S r0[NE];
  for (int e = 0; e < NE; ++e) r0[e] = static_cast<G0S>(g_rest(c[e], s0, m0 * mu[e]));
  vst<G0S, NE>(gptr<G0S>(a.g0_dst) + node * NE, r0);
}

// ---------------------------------------------------------------- k_update
// Occupancy target of the update kernel: three waves per SIMD (at most 168
// VGPRs) where that needs no spilling (float compute, D3Q19 with N <= 5, all
// D2Q9, except the D3Q19 wall variant that collides stored g populations);
// two (at most 256) for the periodic FP64 moment form in D3Q19 with N <= 5;
// otherwise the compiler's own choice.
template <class L, int NC, int ST, bool WALLS = false, int GM = 1>
constexpr int update_waves() {
  if (L::DIM == 3 && WALLS && !GM) return 1;
  if (ST == kStoreF64 && L::DIM == 3 && !WALLS && GM && NC <= 5) return 2;
  return (ST != kStoreF64 && (L::DIM == 2 || NC <= 5)) ? 3 : 1;
}

// LDS planes of the update.  Float with at most four evolved components:
// each position's concentrations form one record of 1, 2 or 4 values (three
// padded to four), read with one vector access at an immediate offset from a
// single base per plane, followed by E_B of every position; otherwise
// field-major (component e of position p at e * PXY + p, then E_B).  Slot
// stride (NEP + 1) PXY.
template <int NE, class T>
constexpr bool update_aos() { return sizeof(T) == 4 && NE <= 4; }
template <int NE, class T>
constexpr int update_nep() { return update_aos<NE, T>() ? (NE == 3 ? 4 : NE) : NE; }

// One workgroup's share of the update: tile b of the simulation (x fastest,
// then y, then the z run), with the LDS window at smem_raw.
// Per-thread diagnostic sums of the reduce mode, internal component order:
// mass, momentum, max |C|, min C, max |sum C - 1|, sum C_c v, sum C_c, and a
// count of nodes with a non-finite field (the record of launch_diag).
template <int NC>
struct DiagAcc {
  double mass[NC], mom[3], maxabs[NC], minc[NC], maxdev, cv[3], cm, nan;
};

// GM: storage of g and f, 0 populations of both, 1 the moment form of g
// (node records C, mu~, v, -3/2 v.v), 2 the moment form of g and the
// record form of f ((fB, F) per node; the reconstruction supplies the
// moments of the streamed f).
template <class L, int NC, int ST, int MODE, bool WALLS, int TXL, int GM>
__device__ __forceinline__ void update_tile(const StepArgs& a,
                                            const DevParams<typename StoreT<ST>::T>* __restrict__ Pp,
                                            int b, unsigned char* smem_raw, DiagAcc<NC>* acc = nullptr) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  constexpr int Q = L::Q;
  constexpr int NE = NC - 1;
  constexpr bool D3 = (L::DIM == 3);
  T* sm = reinterpret_cast<T*>(smem_raw);
  const DevParams<T>* P0 = gptr<const DevParams<T>>(Pp);

  // tile width as a compile-time constant: every LDS access of the stencil
  // is then an immediate offset from one base address
  constexpr int TX = 1 << TXL;
  constexpr int TY = 256 >> TXL;
  constexpr int PX = TX + 2;
  constexpr int PXY = PX * (TY + 2);
  constexpr bool UAOS = update_aos<NE, T>();
  constexpr int NEP = update_nep<NE, T>();
  constexpr int CW = UAOS ? NEP : 1;        // distance between positions' C
  constexpr int CE = UAOS ? 1 : PXY;        // distance between components
  constexpr int EOFF = NEP * PXY;           // E_B of the slot's positions
  constexpr int plane_stride = (NEP + 1) * PXY;
  static_assert(!UAOS || plane_stride % NEP == 0, "LDS records must stay aligned to their size");
  const int tid = threadIdx.x;
  const int tx = tid & (TX - 1);
  const int ty = tid >> TXL;
  // C of the evolved components at a position's C entry (AoS: one record)
  auto read_c = [&](const T* p, T (&o)[NEP]) {
    if constexpr (UAOS) {
      vld<T, NEP>(p, o);
    } else {
#pragma unroll
      for (int e = 0; e < NE; ++e) o[e] = p[e * CE];
    }
  };
  auto write_c = [&](T* p, const T (&v)[NEP]) {
    if constexpr (UAOS) {
      vst<T, NEP>(p, v);
    } else {
#pragma unroll
      for (int e = 0; e < NE; ++e) p[e * CE] = v[e];
    }
  };

  const int tile_x = a.tile_x0 + (b % a.tiles_x) * a.tile_xstep;
  b /= a.tiles_x;
  const int tile_y = b % a.tiles_y;
  const int chunk = b / a.tiles_y;
  const int x0 = tile_x * TX, y0 = tile_y * TY;
  const int z0 = chunk * a.zchunk;
  const int z1 = min(z0 + a.zchunk, a.nz);
  const int x = x0 + tx, y = y0 + ty;
  const bool active = (x < a.nx) && (y < a.ny);
  const size_t n = static_cast<size_t>(a.n);
  const uint32_t nx = a.nx, nxy = uint32_t(a.nx) * uint32_t(a.ny);
  const T* conc = gptr<const T>(a.conc);
  const T* eb = gptr<const T>(a.eb);
  const FS* fsrc = gptr<const FS>(a.f_src);
  // open faces (velocity and concentration Dirichlet); null and 0 otherwise
  const FaceBC<T>* FB = gptr<const FaceBC<T>>(a.faces);
  const int open = (WALLS && FB) ? FB->open : 0;
  auto plain = [&](int face) { return !((open >> face) & 1); };   // a wall face

  // Each thread fills at most two positions of the (TX+2) x (TY+2) LDS window
  // of every plane; their in-plane node offsets are fixed for the workgroup.
  // A position beyond an open face holds the face's values (fill_face).
  uint32_t fill_off[2];
  bool fill_ok[2];
  int fill_face[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int idx = tid + 256 * r;
    fill_ok[r] = idx < PXY;
    fill_off[r] = 0;
    fill_face[r] = -1;
    if (fill_ok[r]) {
      const int ly = idx / PX;
      const int lx = idx - ly * PX;
      int gx = x0 + lx - 1, gy = y0 + ly - 1;
      if (gx < 0 || gx >= a.nx) {
        if (WALLS && a.wall_x) {
          const int face = gx < 0 ? 0 : 1;
          if (plain(face)) fill_ok[r] = false;
          else fill_face[r] = face;
          gx = 0;
        } else {
          gx = wrap(gx, a.nx);
        }
      }
      if (gy < 0 || gy >= a.ny) {
        if (WALLS && a.wall_y) {
          const int face = gy < 0 ? 2 : 3;
          if (plain(face)) fill_ok[r] = false;
          else if (fill_face[r] < 0) fill_face[r] = face;
          gy = 0;
        } else {
          gy = wrap(gy, a.ny);
        }
      }
      fill_off[r] = uint32_t(gx) + nx * uint32_t(gy);
      // beyond an outflow face on x or y: the position's in-plane offset
      // along the other in-plane axis (z is added per plane)
      if (WALLS && fill_ok[r] && fill_face[r] >= 0 && fill_face[r] == a.out_face)
        fill_off[r] = (fill_face[r] >> 1) == 0 ? uint32_t(gy) : uint32_t(gx);
    }
  }

  // C (evolved components) and E_B of plane gz at this thread's fill
  // positions, into registers (fetch_plane), then into an LDS slot
  // (put_plane).  Positions inside a wall are left unfilled: the stencil
  // never reads them.  A position beyond an open face takes the face's
  // values, beyond the outflow face the convected ghost values.
  T nxt[2][NEP + 1];
  bool nok[2];
  auto fetch_plane = [&](int gz) {
    int plane_face = -1;
    bool skip = false;
    if (gz < 0 || gz >= a.nz) {
      if (WALLS && a.wall_z) {
        plane_face = gz < 0 ? 4 : 5;
        skip = plain(plane_face);
        gz = 0;
      } else {
        gz = (gz < 0) ? gz + a.nz : gz - a.nz;
      }
    }
    const uint32_t zoff = uint32_t(gz) * nxy;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      nok[r] = fill_ok[r] && !skip;
      if (!nok[r]) continue;
#pragma unroll
      for (int e = NE; e < NEP; ++e) nxt[r][e] = T(0);
      const int face = fill_face[r] >= 0 ? fill_face[r] : plane_face;
      if (WALLS && face >= 0) {
        if (face == a.out_face) {
          const uint32_t PL = outflow_plane_size(face, a.nx, a.ny, a.nz);
          const uint32_t p = (face >> 1) == 2 ? fill_off[r]
                                              : fill_off[r] + uint32_t((face >> 1) == 0 ? a.ny : a.nx) * uint32_t(gz);
          const T* gh = gptr<const T>(a.out_ghost);
#pragma unroll
          for (int e = 0; e <= NE; ++e) nxt[r][e == NE ? NEP : e] = gh[uint32_t(e) * PL + p];
          continue;
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) nxt[r][e] = FB->cb[face][e];
        nxt[r][NEP] = FB->eb[face];
        continue;
      }
      const uint32_t node = fill_off[r] + zoff;
      vld<T, NE>(at(conc, node * NE), reinterpret_cast<T(&)[NE]>(nxt[r]));
      nxt[r][NEP] = *at(eb, node);
    }
  };
  auto put_plane = [&](int slot) {
    T* base = sm + slot * plane_stride;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!nok[r]) continue;
      const int idx = tid + 256 * r;
      write_c(base + idx * CW, reinterpret_cast<const T(&)[NEP]>(nxt[r]));
      base[EOFF + idx] = nxt[r][NEP];
    }
  };
  auto load_plane = [&](int slot, int gz) {
    fetch_plane(gz);
    put_plane(slot);
  };

  // post-streaming f of this node, gathered from the upstream neighbours, as
  // raw stored numbers (the value times S::scale): the moments unscale once,
  // and the collision forms the raw numbers it stores directly
  T f[Q];
  constexpr T FSC = static_cast<T>(S::scale);
  constexpr T FINV = T(1) / FSC;
  auto load_f = [&](int z) {
    if constexpr (WALLS) {
      // convective outflow: plane N's post-streaming f is in the plane buffer
      const int op = a.out_face >= 0 ? outflow_plane_index(a.out_face, 0, x, y, z, a) : -1;
      if (op >= 0) {
        const uint32_t PL = outflow_plane_size(a.out_face, a.nx, a.ny, a.nz);
        const T* of = gptr<const T>(a.out_f);
#pragma unroll
        for (int k = 1; k < Q; ++k) f[k] = of[uint32_t(k - 1) * PL + op] * FSC;
        return;
      }
    }
    {
      const uint32_t node = uint32_t(x) + nx * uint32_t(y) + nxy * uint32_t(z);
      const Nbr nb = neighbours<L, WALLS>(x, y, z, a);
      const size_t fst = fresh(size_t(a.fstride));
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        if (pulled_from_wall<L, WALLS>(nb, k)) {
          f[k] = S::ld_raw(at(fsrc + size_t(opposite(k) - 1) * fst, node), 0);
          // open face: velocity Dirichlet, bounce-back plus 2 w_k (e_k . v_b) / c_s^2
          const int fc = entry_face<L, WALLS>(nb, k, open);
          if (fc >= 0) f[k] += FB->fcorr[fc][k] * FSC;
        } else {
          f[k] = S::ld_raw(at(fsrc + size_t(k - 1) * fst, upstream<L>(nb, k)), 0);
        }
      }
    }
  };

  // PL (std::true_type): the run has no stabilising term, the conservative
  // force and hydrodynamics, so those flags are not tested per node
  auto process = [&](int z, int s_dn, int s_c, int s_up, auto PL) {
    constexpr bool PLAIN = decltype(PL)::value;
    const bool omega = !PLAIN && (a.flags & kFlagOmega);
    const bool potential = !PLAIN && (a.flags & kFlagPotential);
    // the coefficient tables as seen from this plane: their loads take
    // immediate offsets from one base instead of hoisted per-entry addresses
    const NFLBM_CONST DevParams<T>& P = *fresh_const(P0);
    const int li = (ty + 1) * PX + (tx + 1);
    // solid geometry: this node's pull mask (bit k: the neighbour x - e_k is
    // solid or beyond a wall face; bit 0: this node is solid)
    bool geom = false;
    uint32_t pm = 0u;
    if constexpr (WALLS) {
      if (a.bb) {
        geom = true;
        pm = a.bb[uint32_t(x) + nx * uint32_t(y) + nxy * uint32_t(z)];
      }
    }
    // record form of f in a step: the moments of the streamed f are read
    // here, so that the load's latency passes under the stencil (four
    // registers, where the gathered populations would hold eighteen)
    constexpr bool FM_EARLY = GM == 2 && MODE == kModeStep;
    T fm_early[4];
    if constexpr (FM_EARLY)
      rec_load<S, 4>(a.fmom, (uint32_t(x) + nx * uint32_t(y) + nxy * uint32_t(z)) * 4u, fm_early, T(S::vel_scale));
    // Per-plane LDS bases of the 3 x 3 neighbourhood's lowest corner (C and
    // E_B entries of the slots below, at and above), made opaque here so
    // that every stencil read is one of them plus an immediate offset
    // rather than a hoisted per-neighbour address plus the slot's base.
    auto opaque = [](uint32_t v) {
      asm volatile("" : "+v"(v));
      return v;
    };
    const uint32_t corner_c = uint32_t((li - PX - 1) * CW), corner_e = uint32_t(EOFF + li - PX - 1);
    const uint32_t bc[3] = {D3 ? opaque(uint32_t(s_dn * plane_stride) + corner_c) : 0u,
                            opaque(uint32_t(s_c * plane_stride) + corner_c),
                            D3 ? opaque(uint32_t(s_up * plane_stride) + corner_c) : 0u};
    const uint32_t be[3] = {D3 ? opaque(uint32_t(s_dn * plane_stride) + corner_e) : 0u,
                            opaque(uint32_t(s_c * plane_stride) + corner_e),
                            D3 ? opaque(uint32_t(s_up * plane_stride) + corner_e) : 0u};
    T c[NC];
    {
      T cr[NEP];
      read_c(sm + bc[1] + (PX + 1) * CW, cr);
      T rest = cr[0];
      c[0] = cr[0];
#pragma unroll
      for (int e = 1; e < NE; ++e) {
        c[e] = cr[e];
        rest += c[e];
      }
      c[NE] = T(1) - rest;
    }
    const T E0 = sm[be[1] + PX + 1];
    T gC[NC][3];
    T lap[NC];
    T gE[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      lap[i] = T(0);
      gC[i][0] = gC[i][1] = gC[i][2] = T(0);
    }
    // ---- isotropic stencils (Eq. gradstencil and the Laplacian after it).
    // From the lowest corner of the 3 x 3 neighbourhood every LDS offset is a
    // non-negative immediate.
    auto nbr = [&](int ex, int ey, int ez) {      // C entry of x + e
      return sm + bc[ez + 1] + ((1 + ey) * PX + (1 + ex)) * CW;
    };
    auto nbr_e = [&](int ex, int ey, int ez) {    // E_B of x + e
      return sm + be[ez + 1] + (1 + ey) * PX + (1 + ex);
    };
    // A node next to a wall face goes direction by direction; every other
    // node, in every kernel variant and tile shape alike, goes by pairs, so a
    // node's result depends only on its position.
    bool near_wall = false;
    if constexpr (WALLS) {
      near_wall = geom ? (pm >> 1) != 0u
                       : (a.wall_x && ((x == 0 && plain(0)) || (x == a.nx - 1 && plain(1)))) ||
                             (a.wall_y && ((y == 0 && plain(2)) || (y == a.ny - 1 && plain(3)))) ||
                             (a.wall_z && ((z == 0 && plain(4)) || (z == a.nz - 1 && plain(5))));
    }
    if (!near_wall) {
      // over the opposite pairs {k, k+1}, with psi+ = psi(x + e_k) and
      // psi- = psi(x - e_k) the gradient takes w_k e_k (psi+ - psi-) and the
      // Laplacian w_k (psi+ + psi-), less (sum of the moving weights) psi(x)
      // at the end: a tenth fewer instructions than direction by direction
#pragma unroll
      for (int k = 1; k < Q; k += 2) {
        const int ex = L::e[k][0], ey = L::e[k][1], ez = L::e[k][2];
        const T wk = static_cast<T>(L::w[k]);
        T rp[NEP], rm[NEP];
        read_c(nbr(ex, ey, ez), rp);
        read_c(nbr(-ex, -ey, -ez), rm);
#pragma unroll
        for (int i = 0; i < NE; ++i) {
          const T vp = rp[i], vm = rm[i];
          const T dd = vp - vm;
          lap[i] = fma(wk, vp + vm, lap[i]);
          if (ex != 0) gC[i][0] = fma((ex > 0) ? wk : -wk, dd, gC[i][0]);
          if (ey != 0) gC[i][1] = fma((ey > 0) ? wk : -wk, dd, gC[i][1]);
          if (ez != 0) gC[i][2] = fma((ez > 0) ? wk : -wk, dd, gC[i][2]);
        }
        const T dE = *nbr_e(ex, ey, ez) - *nbr_e(-ex, -ey, -ez);
        if (ex != 0) gE[0] = fma((ex > 0) ? wk : -wk, dE, gE[0]);
        if (ey != 0) gE[1] = fma((ey > 0) ? wk : -wk, dE, gE[1]);
        if (ez != 0) gE[2] = fma((ez > 0) ? wk : -wk, dE, gE[2]);
      }
      constexpr T wsum = moving_weight_sum<L, T>();
#pragma unroll
      for (int i = 0; i < NE; ++i) lap[i] = fma(-wsum, c[i], lap[i]);
    } else {
      // next to a wall, direction by direction: a neighbour inside a wall
      // takes the centre value, i.e. contributes nothing
      Nbr nbw;
      if (geom && open) nbw = neighbours<L, WALLS>(x, y, z, a);
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        const int ex = L::e[k][0], ey = L::e[k][1], ez = L::e[k][2];
        const T wk = static_cast<T>(L::w[k]);
        bool wall = false;
        if (geom) {
          wall = (pm >> opposite(k)) & 1u;      // x + e_k is x - e_(opposite k)
          // beyond an open face (not continuing a solid node): an ordinary
          // LDS position holding the face's values
          if (wall && open && entry_face<L, WALLS>(nbw, opposite(k), open) >= 0) wall = false;
        } else {
          // a neighbour beyond an open face is an ordinary LDS position
          if (ex != 0 && a.wall_x) wall |= (x + ex < 0 && plain(0)) || (x + ex >= a.nx && plain(1));
          if (ey != 0 && a.wall_y) wall |= (y + ey < 0 && plain(2)) || (y + ey >= a.ny && plain(3));
          if (ez != 0 && a.wall_z) wall |= (z + ez < 0 && plain(4)) || (z + ez >= a.nz && plain(5));
        }
        if (!wall) {
          T rn[NEP];
          read_c(nbr(ex, ey, ez), rn);
#pragma unroll
          for (int i = 0; i < NE; ++i) {
            const T d = rn[i] - c[i];
            lap[i] = fma(wk, d, lap[i]);
            if (ex != 0) gC[i][0] = fma((ex > 0) ? wk : -wk, d, gC[i][0]);
            if (ey != 0) gC[i][1] = fma((ey > 0) ? wk : -wk, d, gC[i][1]);
            if (ez != 0) gC[i][2] = fma((ez > 0) ? wk : -wk, d, gC[i][2]);
          }
          const T dE = *nbr_e(ex, ey, ez) - E0;
          if (ex != 0) gE[0] = fma((ex > 0) ? wk : -wk, dE, gE[0]);
          if (ey != 0) gE[1] = fma((ey > 0) ? wk : -wk, dE, gE[1]);
          if (ez != 0) gE[2] = fma((ez > 0) ? wk : -wk, dE, gE[2]);
        }
      }
    }
    // the implicit component is 1 - sum of the others, so each of its stencil
    // differences is minus the sum of theirs
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      lap[NE] -= lap[i];
#pragma unroll
      for (int d = 0; d < 3; ++d) gC[NE][d] -= gC[i][d];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      lap[i] *= T(6);
#pragma unroll
      for (int d = 0; d < 3; ++d) gC[i][d] *= T(3);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) gE[d] *= T(3);

    // ---- flux potential mu~ of the evolved components (factored form)
    T mu[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      T br = -(T(1) - T(3) * c[i] + T(2) * c[i] * c[i]);
#pragma unroll
      for (int l = 0; l < NC; ++l) {
        if (l == i) continue;
        // rows with no term are skipped at compile time (a zero row would
        // still cost an instruction: 0 times c[l] is not folded away)
        T row = T(0);
        bool any = false;
#pragma unroll
        for (int m = l + 1; m < NC; ++m)
          if (m != i) {
            row = any ? fma(P.psi[i][l][m], c[m], row) : P.psi[i][l][m] * c[m];
            any = true;
          }
        if (any) br = fma(row, c[l], br);
      }
      T val = fma(P.k34D, lap[i], (P.k12D * c[i]) * br);
      if (omega) {
        T sx = T(0);
#pragma unroll
        for (int k2 = 0; k2 < NC; ++k2)
#pragma unroll
          for (int l = k2 + 1; l < NC; ++l)
            if (k2 != i && l != i) sx = fma(P.xt[i][k2][l], (c[k2] * c[k2]) * (c[l] * c[l]), sx);
        T sy = T(0);
#pragma unroll
        for (int l = 0; l < NC; ++l) {
          if (l == i) continue;
          T inner = T(0);
#pragma unroll
          for (int m = 0; m < NC; ++m)
            if (m != i && m != l) inner = fma(P.zt[i][l][m], c[m], inner);
          sy = fma(c[l] * c[l], inner, sy);
        }
        val = fma((P.k12D * P.omega_stab) * c[i], fma(c[i], sy, sx), val);
      }
      mu[i] = val;
    }
    // NaN check, first half: a non-finite C or mu~ makes t - t NaN (finite
    // values give 0); taken here so that mu~ need not live any longer
    bool bad = false;
    if (MODE == kModeStep && (a.flags & kFlagCheckNaN)) {
      T t = T(0);
#pragma unroll
      for (int i = 0; i < NE; ++i) t += c[i] + mu[i];
      bad = !(t - t == T(0));
    }
    if constexpr (GM >= 1 && MODE == kModeStep) {
      // moment form: mu~ goes to the node record at once instead of being
      // held through the gather of f
      const uint32_t nd = uint32_t(x) + nx * uint32_t(y) + nxy * uint32_t(z);
      rec_store<S, NE, true>(a.mu, nd * NE, mu, T(S::mu_scale));
    }

    // ---- surface tension force (Eq. Fsnew, or Eq. ststand) + body force
    T F[3];
    if (potential) {
      F[0] = F[1] = F[2] = T(0);
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        T mraw = T(0);
#pragma unroll
        for (int k2 = 0; k2 < NC; ++k2)
          if (k2 != i)
            mraw += fma(P.kappa[i][k2], lap[k2], P.beta[i][k2] * (fprime(c[i]) - fprime(c[i] + c[k2])));
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] = fma(mraw, gC[i][d], F[d]);
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
          if (j != i) kl = fma(P.kappa[i][j], lap[j], kl);
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] = fma(kl, gC[i][d], F[d]);
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] += P.fb[d];

    // ---- hydrodynamic moments (Eqs. nmom, pres with rho = 1).  f is gathered
    // only now: loading it before the stencil would keep Q-1 more registers
    // live through it and cost occupancy.
    const uint32_t node = uint32_t(x) + nx * uint32_t(y) + nxy * uint32_t(z);
    // diffusive-only runs (Sec. IV B) do not evolve f: v = 0 and P = 0
    const bool hydro = PLAIN || !(a.flags & kFlagNoHydro);
    // Over the opposite pairs {k, k+1}: sp = f_k + f_k+1 and dp = f_k - f_k+1
    // give the moments (sum_k f_k and sum_k e_k f_k) and, below, the even and
    // odd parts the TRT collision relaxes; f itself is not needed after this.
    constexpr int NP = Q / 2;
    T sp[NP], dp[NP];
    T v[3] = {T(0), T(0), T(0)};
    T fsum = T(0);
#pragma unroll
    for (int p = 0; p < NP; ++p) sp[p] = dp[p] = T(0);
    // record form of f: the reconstruction has formed sum_k f_k and
    // sum_k e_k f_k of the streamed f (the read-back modes see the form at
    // run time)
    const bool frec = GM == 2 || (GM == 0 && MODE != kModeStep && (a.flags & kFlagFRecord));
    if (hydro && frec) {
      T fm[4];
      if constexpr (FM_EARLY) {
#pragma unroll
        for (int d = 0; d < 4; ++d) fm[d] = fm_early[d];
      } else {
        rec_load<S, 4>(a.fmom, node * 4, fm, T(S::vel_scale));
      }
      fsum = fm[0];
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] = fma(T(0.5), F[d], fm[1 + d]);
    } else if (hydro && GM != 2) {
      load_f(z);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int k = 2 * p + 1;
        sp[p] = f[k] + f[k + 1];
        dp[p] = f[k] - f[k + 1];
        fsum += sp[p];
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (L::e[k][d] != 0) v[d] += (L::e[k][d] > 0) ? dp[p] : -dp[p];
      }
      fsum *= FINV;
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] = fma(T(0.5), F[d], v[d] * FINV);
    }
    const T vv = fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0]));
    const T s0 = static_cast<T>(L::w[0]) * (-T(1.5) * vv);
    const T Pn = static_cast<T>((1.0 / 3.0) / (1.0 - L::w[0])) * (fsum + s0);

    if constexpr (MODE == kModeFields) {
      double* out = gptr<double>(a.fields);
      if (pm & 1u) {          // a solid node: no fluid, every field 0
#pragma unroll
        for (int r = 0; r < 2 * NC + 7; ++r) out[size_t(r) * n + node] = 0.0;
        return;
      }
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
    if constexpr (MODE == kModeReduce) {
      // the FP64 fields of this node, as the fields mode writes them, summed
      // into the thread's diagnostics; solid nodes hold no fluid
      if (pm & 1u) return;
      DiagAcc<NC>& A = *acc;
      double csum = 0.0, probe = 0.0;
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        const double ci = static_cast<double>(c[i]);
        A.mass[i] += ci;
        A.maxabs[i] = fmax(A.maxabs[i], fabs(ci));
        A.minc[i] = fmin(A.minc[i], ci);
        csum += ci;
        probe += ci * 0.0;
        if (i < NE) probe += static_cast<double>(mu[i]) * 0.0;
      }
      A.maxdev = fmax(A.maxdev, fabs(csum - 1.0));
      double cc = 0.0;
#pragma unroll
      for (int i = 0; i < NC; ++i)
        if (i == a.diag_vcm) cc = static_cast<double>(c[i]);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double vd = static_cast<double>(v[d]);
        A.mom[d] += vd;
        A.cv[d] += cc * vd;
        probe += vd * 0.0 + static_cast<double>(F[d]) * 0.0;
      }
      A.cm += cc;
      probe += static_cast<double>(Pn) * 0.0;
      A.nan += (probe == 0.0) ? 0.0 : 1.0;
      return;
    }
    if (a.flags & kFlagCheckNaN) {
      // second half: v and P
      const T t = vv + Pn;
      if (bad || !(t - t == T(0))) *a.nanflag = 1;
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

    FS* fdst = gptr<FS>(a.f_dst);
    FS* gkdst = gptr<FS>(a.gk_dst);
    G0S* g0dst = gptr<G0S>(a.g0_dst);
    const FS* gksrc = gptr<const FS>(a.gk_src);
    const T base_s = -T(1.5) * vv;
    if constexpr (GM >= 1) {
      // moment form: the reconstruction re-forms g* from mu~ (stored above),
      // v and -3/2 v.v
      const T vel[4] = {v[0], v[1], v[2], base_s};
      rec_store<S, 4, true>(a.vel, node * 4, vel, T(S::vel_scale));
    }
    const T vF = fma(v[2], F[2], fma(v[1], F[1], v[0] * F[0]));
    const T cP = T(3) * Pn;
    if constexpr (GM == 2) {
      // record form of f: with omega+ = omega- = 1 the collision leaves
      // f*_k = w_k [s_k / w_k + fB + (e.F)(9/2 e.v +- 3/2)] (see f_scaled),
      // so the node stores fB = 3 P - 3/2 v.F and F beside (v, -3/2 v.v)
      const T fr[4] = {static_cast<T>(fma(-T(1.5), vF, cP)), F[0], F[1], F[2]};
      rec_store<S, 4, true>(a.frec, node * 4, fr, T(S::vel_scale));
      return;
    }
    // Per-node factors of the pair collision.  With s = f_k + f_k+1,
    // d = f_k - f_k+1, e_k.v and e_k.F of the odd member k, the TRT step with
    // Guo forcing (Eqs. TRT, FTRT, hydroforce) is, in exact arithmetic,
    //   f*_k = S + D,  f*_k+1 = S - D,
    //   S = (1 - w+)/2 s + w_k [w+ (3P + 4.5 (e.v)^2 - 1.5 v.v) + (1 - w+/2)(9 (e.v)(e.F) - 3 v.F)]
    //   D = (1 - w-)/2 d + w_k [3 w- e.v + 3 (1 - w-/2) e.F]
    // i.e. the even and odd parts relax towards those of f^eq and take those
    // of F_k, with the equilibrium and force pair terms written out.
    const T A3 = cP + base_s;
    const T B3 = -T(3) * vF;
    const T hp2 = fma(-T(0.5), wp, T(1));
    const T hm6 = T(3) * fma(-T(0.5), wm, T(1));
    const T wm3 = T(3) * wm;
    const T cs = T(0.5) * (T(1) - wp);
    const T cd = T(0.5) * (T(1) - wm);
    T moved[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) moved[i] = T(0);
    Nbr nb;
    if (GM == 0 && (a.flags & kFlagNeedG)) nb = neighbours<L, WALLS>(x, y, z, a);
    const size_t fst = fresh(size_t(a.fstride));
    const size_t gst = fresh(size_t(a.gstride));
    // convective outflow: plane N's post-streaming g is in the plane buffer
    int gop = -1;
    uint32_t gPL = 0;
    if (WALLS && GM == 0 && (a.flags & kFlagNeedG) && a.out_face >= 0) {
      gop = outflow_plane_index(a.out_face, 0, x, y, z, a);
      gPL = outflow_plane_size(a.out_face, a.nx, a.ny, a.nz);
    }

    // ---- per direction pair: TRT collision of f with forcing and BGK
    // collision of every evolved g; stores go to this node (pull layout)
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
      const int kb = k + 1;
      const int p = k >> 1;
      const T wk = static_cast<T>(L::w[k]);
      const T ev = proj<L>(k, v), eF = proj<L>(k, F);
      if (hydro) {
        const T q = fma(T(4.5) * ev, ev, A3);
        const T fo = fma(T(9) * ev, eF, B3);
        const T Is = fma(hp2, fo, wp * q);
        const T Ia = fma(hm6, eF, wm3 * ev);
        // sp, dp are raw: S and D come out raw too, with w_k scaled
        const T Sx = fma(cs, sp[p], (wk * FSC) * Is);
        const T Dx = fma(cd, dp[p], (wk * FSC) * Ia);
        st_nt(at(fdst + size_t(k - 1) * fst, node), S::pack_raw(Sx + Dx));
        st_nt(at(fdst + size_t(kb - 1) * fst, node), S::pack_raw(Sx - Dx));
      }
      if constexpr (GM >= 1) continue;
      const T quad = quad_term<L>(ev, base_s);
      const T sk_k = s_pair_member<L>(k, ev, quad);
      const T sk_b = s_pair_member<L>(kb, ev, quad);
      const T mw = wk * P.m;
      FS qk[NE], qb[NE];
      FS ok[NE], ob[NE];
      // open faces: the pulled g are anti-bounced (see the reconstruction)
      int fk = -1, fb = -1;
      if (WALLS && open && (a.flags & kFlagNeedG)) {
        fk = entry_face<L, WALLS>(nb, k, open);
        fb = entry_face<L, WALLS>(nb, kb, open);
      }
      if (a.flags & kFlagNeedG) {
        if (pulled_from_wall<L, WALLS>(nb, k))
          vld<FS, NE>(at(gksrc + size_t(kb - 1) * gst, node * NE), ok);
        else
          vld<FS, NE>(at(gksrc + size_t(k - 1) * gst, upstream<L>(nb, k) * NE), ok);
        if (pulled_from_wall<L, WALLS>(nb, kb))
          vld<FS, NE>(at(gksrc + size_t(k - 1) * gst, node * NE), ob);
        else
          vld<FS, NE>(at(gksrc + size_t(kb - 1) * gst, upstream<L>(nb, kb) * NE), ob);
      }
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const T mmu = mw * mu[i];
        T gk = fma(c[i], sk_k, -mmu);
        T gb = fma(c[i], sk_b, -mmu);
        if (a.flags & kFlagNeedG) {
          T o1 = S::unpack(ok[i]), o2 = S::unpack(ob[i]);
          if (fk >= 0) o1 = FB->gsum[fk][i][k] - o1;
          if (fb >= 0) o2 = FB->gsum[fb][i][kb] - o2;
          if (WALLS && gop >= 0) {
            const T* og = gptr<const T>(a.out_g);
            o1 = og[(uint32_t(i) * Q + k) * gPL + gop];
            o2 = og[(uint32_t(i) * Q + kb) * gPL + gop];
          }
          gk = o1 - (o1 - gk) * P.inv_tau_g[i];
          gb = o2 - (o2 - gb) * P.inv_tau_g[i];
        }
        qk[i] = S::pack(gk);
        qb[i] = S::pack(gb);
        moved[i] += S::unpack(qk[i]) + S::unpack(qb[i]);
      }
      vst_nt<FS, NE>(at(gkdst + size_t(k - 1) * gst, node * NE), qk);
      vst_nt<FS, NE>(at(gkdst + size_t(kb - 1) * gst, node * NE), qb);
    }
    if constexpr (GM == 0) {
      G0S r0[NE];
#pragma unroll
      for (int i = 0; i < NE; ++i) r0[i] = static_cast<G0S>(c[i] - moved[i]);
      vst_nt<G0S, NE>(at(g0dst, node * NE), r0);
    }
  };

  auto march = [&](auto PL) {
    if constexpr (D3 && sizeof(T) == 4) {
      // Float: rolling window of three LDS planes, with the next plane's
      // values fetched into registers while the current plane is processed
      // and written to LDS at the top of the next iteration, so that the
      // fill's load latency overlaps the compute.
      load_plane(0, z0 - 1);
      load_plane(1, z0);
      fetch_plane(z0 + 1);
      for (int z = z0; z < z1; ++z) {
        const int r = z - z0;
        const int s_dn = r % 3, s_c = (r + 1) % 3, s_up = (r + 2) % 3;
        asm volatile("" ::: "memory");
        put_plane(s_up);
        __syncthreads();
        if (z + 1 < z1) fetch_plane(z + 2);
        if (active) process(z, s_dn, s_c, s_up, PL);
        __syncthreads();
      }
    } else if constexpr (D3) {
      // rolling window of three LDS planes: z-1, z, z+1
      load_plane(0, z0 - 1);
      load_plane(1, z0);
      for (int z = z0; z < z1; ++z) {
        const int r = z - z0;
        const int s_dn = r % 3, s_c = (r + 1) % 3, s_up = (r + 2) % 3;
        // keep the per-plane coefficient loads inside the loop (scalar cache
        // hits) instead of holding every coefficient live across all planes
        asm volatile("" ::: "memory");
        load_plane(s_up, z + 1);
        __syncthreads();
        if (active) process(z, s_dn, s_c, s_up, PL);
        __syncthreads();
      }
    } else {
      load_plane(0, 0);
      __syncthreads();
      if (active) process(0, 0, 0, 0, PL);
    }
  };
  if constexpr (MODE == kModeStep) {
    if (!(a.flags & (kFlagOmega | kFlagPotential | kFlagNoHydro))) march(std::true_type{});
    else march(std::false_type{});
  } else {
    march(std::false_type{});
  }
}

template <class L, int NC, int ST, int MODE, bool WALLS, int TXL, int GM>
__global__ void __launch_bounds__(256, (update_waves<L, NC, ST, WALLS, GM>()))
k_update(StepArgs a, const DevParams<typename StoreT<ST>::T>* __restrict__ Pp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nblocks = a.tiles_x * a.tiles_y * a.chunks_z;
  if constexpr (MODE == kModeReduce) {
    // grid-stride over the tiles (the grid is capped, so the partial records
    // take bounded memory), then one record per workgroup
    DiagAcc<NC> acc;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      acc.mass[i] = acc.maxabs[i] = 0.0;
      acc.minc[i] = 1e300;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) acc.mom[d] = acc.cv[d] = 0.0;
    acc.maxdev = acc.cm = acc.nan = 0.0;
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
      update_tile<L, NC, ST, MODE, WALLS, TXL, GM>(a, Pp, b, smem_raw, &acc);
      __syncthreads();
    }
    double* scratch = reinterpret_cast<double*>(smem_raw);
    double* out = gptr<double>(a.diag_partial) + size_t(blockIdx.x) * (3 * NC + 9);
    auto put = [&](int q, double v, int op) {
      v = block_reduce_d(v, op, scratch);
      if (threadIdx.x == 0) out[q] = v;
    };
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      put(i, acc.mass[i], 0);
      put(NC + 3 + i, acc.maxabs[i], 1);
      put(2 * NC + 3 + i, acc.minc[i], 2);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      put(NC + d, acc.mom[d], 0);
      put(3 * NC + 4 + d, acc.cv[d], 0);
    }
    put(3 * NC + 3, acc.maxdev, 1);
    put(3 * NC + 7, acc.cm, 0);
    put(3 * NC + 8, acc.nan, 0);
  } else {
    update_tile<L, NC, ST, MODE, WALLS, TXL, GM>(a, Pp, xcd_remap(static_cast<int>(blockIdx.x), nblocks),
                                                 smem_raw);
  }
}

// Batch form (see k_conc_batch).  The work list holds each simulation's
// tiles contiguously, so the XCD remap keeps a simulation's neighbouring tiles
// on one XCD.
template <class L, int NC, int ST, bool WALLS, int TXL, int GM>
__global__ void __launch_bounds__(256, (update_waves<L, NC, ST, WALLS, GM>()))
k_update_batch(const StepArgs* __restrict__ args, const DevParams<typename StoreT<ST>::T>* __restrict__ params,
               const int2* __restrict__ work, int nblocks) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 w = work[xcd_remap(static_cast<int>(blockIdx.x), nblocks)];
  const StepArgs a = args[w.x];
  update_tile<L, NC, ST, kModeStep, WALLS, TXL, GM>(a, params + w.x, w.y, smem_raw);
}

// ------------------------------------------------------------------ k_init
// Writes the post-collision arrays so that the first gather yields
// f_k = f^eq_k(P0, v0) (k >= 1), g_{i,0} = C_i, g_{i,k>=1} = 0: the value a
// node must receive along e_k is stored where that node will pull it from.
// Every slot is written exactly once.  In the moment form the same g follows
// from the record C = C0, mu~ = 0, v = 0 (every s_k(0) is 0).
template <class L, int NC, int ST, bool WALLS, int GM>
__global__ void __launch_bounds__(256) k_init(InitArgs a) {
  using S = StoreT<ST>;
  using T = typename S::T;
  using FS = typename S::FS;
  using G0S = typename S::G0S;
  constexpr int Q = L::Q;
  constexpr int NE = NC - 1;
  const DevParams<T>& P = *static_cast<const DevParams<T>*>(a.params);
  const size_t n = static_cast<size_t>(a.n);
  const size_t fst = static_cast<size_t>(a.sa.fstride), gst = static_cast<size_t>(a.sa.gstride);
  FS* f = static_cast<FS*>(a.f);
  FS* gk = static_cast<FS*>(a.gk);
  G0S* g0 = static_cast<G0S*>(a.g0);
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int z = blockIdx.z;
  if (x >= a.sa.nx || y >= a.sa.ny) return;
  const uint32_t node = uint32_t(x) + uint32_t(a.sa.nx) * (uint32_t(y) + uint32_t(a.sa.ny) * uint32_t(z));
  const Nbr nb = neighbours<L, WALLS>(x, y, z, a.sa);
  if (solid_node<WALLS>(nb)) {
    // no fluid: this node's own stored values are 0 (no fluid node reads them)
    FS zf[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) zf[e] = S::pack(T(0));
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      if (GM != 2) f[size_t(k - 1) * fst + node] = S::pack(T(0));
      if (GM == 0) vst<FS, NE>(gk + size_t(k - 1) * gst + size_t(node) * NE, zf);
    }
    if constexpr (GM == 2) {
      const T zr[4] = {T(0), T(0), T(0), T(0)};
      rec_store<S, 4, false>(a.sa.frec, uint32_t(node) * 4u, zr, T(S::vel_scale));
    }
    T z0[NE], z4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < NE; ++i) z0[i] = T(0);
    if constexpr (GM >= 1) {
      vst<T, NE>(gptr<T>(a.sa.cprev) + size_t(node) * NE, z0);
      rec_store<S, NE, false>(a.sa.mu, uint32_t(node) * uint32_t(NE), z0, T(S::mu_scale));
      rec_store<S, 4, false>(a.sa.vel, uint32_t(node) * 4u, z4, T(S::vel_scale));
    } else {
      G0S g00[NE];
#pragma unroll
      for (int i = 0; i < NE; ++i) g00[i] = G0S(0);
      vst<G0S, NE>(g0 + size_t(node) * NE, g00);
    }
    return;
  }
  double v[3] = {0.0, 0.0, 0.0};
  double Pn = 0.0;
  if (a.v)
    for (int d = 0; d < 3; ++d) v[d] = a.v[size_t(d) * n + node];
  if (a.P) Pn = a.P[node];
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  FS zero[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) zero[e] = S::pack(T(0));
  if constexpr (GM == 2) {
    // record form of f: (A0, v0) with A0 = 3 P0 - 3/2 v0.v0; the first step
    // takes each node's f as this record's equilibrium (kFlagFLocal)
    const T fr[4] = {static_cast<T>(3.0 * Pn - 1.5 * vv), static_cast<T>(v[0]), static_cast<T>(v[1]),
                     static_cast<T>(v[2])};
    rec_store<S, 4, false>(a.sa.frec, uint32_t(node) * 4u, fr, T(S::vel_scale));
  }
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    if constexpr (GM == 2) break;
    double ev = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) ev += L::e[k][d] * v[d];
    const double s = L::w[k] * (3.0 * ev + 4.5 * ev * ev - 1.5 * vv);
    const FS val = S::pack(static_cast<T>(3.0 * L::w[k] * Pn + s));
    if (pulled_from_wall<L, WALLS>(nb, k)) {
      // an open face adds its correction to the slot on the way in: store the
      // value that the first step then reads as f_k = val and g_k = 0
      const FaceBC<T>* FB = gptr<const FaceBC<T>>(a.sa.faces);
      const int fc = entry_face<L, WALLS>(nb, k, (WALLS && FB) ? FB->open : 0);
      if (fc >= 0) {
        f[size_t(opposite(k) - 1) * fst + node] =
            S::pack(static_cast<T>(3.0 * L::w[k] * Pn + s) - FB->fcorr[fc][k]);
        if (GM == 0) {
          FS gs[NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) gs[e] = S::pack(FB->gsum[fc][e][k]);
          vst<FS, NE>(gk + size_t(opposite(k) - 1) * gst + size_t(node) * NE, gs);
        }
        continue;
      }
      f[size_t(opposite(k) - 1) * fst + node] = val;
      if (GM == 0) vst<FS, NE>(gk + size_t(opposite(k) - 1) * gst + size_t(node) * NE, zero);
    } else {
      const uint32_t src = upstream<L>(nb, k);
      f[size_t(k - 1) * fst + src] = val;
      if (GM == 0) vst<FS, NE>(gk + size_t(k - 1) * gst + size_t(src) * NE, zero);
    }
  }
  if constexpr (GM >= 1) {
    T c0[NE], z0[NE], z4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      c0[i] = static_cast<T>(a.C[size_t(P.uidx[i]) * n + node]);
      z0[i] = T(0);
    }
    vst<T, NE>(gptr<T>(a.sa.cprev) + size_t(node) * NE, c0);
    rec_store<S, NE, false>(a.sa.mu, uint32_t(node) * uint32_t(NE), z0, T(S::mu_scale));
    rec_store<S, 4, false>(a.sa.vel, uint32_t(node) * 4u, z4, T(S::vel_scale));
  } else {
    G0S c0[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) c0[i] = static_cast<G0S>(a.C[size_t(P.uidx[i]) * n + node]);
    vst<G0S, NE>(g0 + size_t(node) * NE, c0);
  }
}

// Record form of f: the f the next gather reads, in the population layout
// (compute precision, direction stride a.fstride), for read-back.  After a
// step every node's post-collision f*_k is formed from its records; after
// set_fields (kFlagFLocal) each node's initial equilibrium is placed where
// its first gather pulls it from, as k_init places populations.
template <class L, int ST, bool WALLS>
__global__ void __launch_bounds__(256) k_expand_f(StepArgs a, void* out) {
  using S = StoreT<ST>;
  using T = typename S::T;
  constexpr int Q = L::Q;
  const size_t n = static_cast<size_t>(a.n);
  const size_t node = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (node >= n) return;
  const size_t fst = static_cast<size_t>(a.fstride);
  T* o = static_cast<T*>(out);
  T fr[4];
  rec_load<S, 4>(a.frec, uint32_t(node * 4), fr, T(S::vel_scale));
  if (!(a.flags & kFlagFLocal)) {
    T v4[4];
    rec_load<S, 4>(a.vel, uint32_t(node * 4), v4, T(S::vel_scale));
#pragma unroll
    for (int k = 1; k < Q; ++k) o[size_t(k - 1) * fst + node] = static_cast<T>(L::w[k]) * f_scaled<L>(k, v4, fr);
    return;
  }
  const int x = int(node % size_t(a.nx));
  const int y = int((node / size_t(a.nx)) % size_t(a.ny));
  const int z = int(node / (size_t(a.nx) * size_t(a.ny)));
  const Nbr nb = neighbours<L, WALLS>(x, y, z, a);
  if (solid_node<WALLS>(nb)) {
#pragma unroll
    for (int k = 1; k < Q; ++k) o[size_t(k - 1) * fst + node] = T(0);
    return;
  }
  const FaceBC<T>* FB = gptr<const FaceBC<T>>(a.faces);
  const int open = (WALLS && FB) ? FB->open : 0;
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    T val = static_cast<T>(L::w[k]) * f_scaled_local<L>(k, fr);
    if (pulled_from_wall<L, WALLS>(nb, k)) {
      // across an open face the read-back adds the face's correction
      const int fc = entry_face<L, WALLS>(nb, k, open);
      if (WALLS && fc >= 0) val -= FB->fcorr[fc][k];
      o[size_t(opposite(k) - 1) * fst + node] = val;
    } else {
      o[size_t(k - 1) * fst + upstream<L>(nb, k)] = val;
    }
  }
}

// ---------------------------------------------------------------- k_reduce
#if !defined(NFLBM_UNIT_STORE) || NFLBM_UNIT_STORE < 0
// Diagnostic record: mass[N], mom[3], maxabs[N], minc[N], maxdev, cv[3], cmass, nan.
__host__ __device__ int reduce_record_len(int N) { return 3 * N + 9; }

// ------------------------------------------------------------ solid geometry
// StepArgs::bb of every node from the byte mask solid[n]: bit k set when
// x - e_k lies beyond a wall face or is solid, bit 0 when x is solid.
template <class L>
__global__ void __launch_bounds__(256) k_build_bb(const unsigned char* __restrict__ solid,
                                                  uint32_t* __restrict__ bb, StepArgs a) {
  const size_t n = static_cast<size_t>(a.n);
  const size_t node = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (node >= n) return;
  const int x = int(node % size_t(a.nx));
  const int y = int((node / size_t(a.nx)) % size_t(a.ny));
  const int z = int(node / (size_t(a.nx) * size_t(a.ny)));
  const int dims[3] = {a.nx, a.ny, a.nz};
  const int walls[3] = {a.wall_x, a.wall_y, a.wall_z};
  uint32_t m = solid[node] ? 1u : 0u;
  for (int k = 1; k < L::Q; ++k) {
    int c[3] = {x - L::e[k][0], y - L::e[k][1], z - L::e[k][2]};
    bool blocked = false;
    for (int d = 0; d < 3; ++d) {
      if (c[d] < 0 || c[d] >= dims[d]) {
        if (walls[d]) blocked = true;
        c[d] = (c[d] + dims[d]) % dims[d];
      }
    }
    if (!blocked) blocked = solid[size_t(c[0]) + size_t(a.nx) * (size_t(c[1]) + size_t(a.ny) * size_t(c[2]))] != 0;
    if (blocked) m |= 1u << k;
  }
  bb[node] = m;
}

// ------------------------------------------------------------ domain size
// lambda_i = H(C_i - 1/2) of every component from the fields-mode C [N][n].
__global__ void __launch_bounds__(256) k_lambda(const double* __restrict__ C, double* __restrict__ lam,
                                                long long total) {
  const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
  if (i < total) lam[i] = C[i] > 0.5 ? 1.0 : 0.0;
}

// Partial sums of S(k) = |X(k)|^2 and |k| S(k) over the half spectrum of an
// R2C transform (nz x ny x (nx/2 + 1) per component, component blockIdx.y),
// k = 0 left out; wave vectors kept once stand for their conjugates too.
__global__ void __launch_bounds__(256) k_spectrum(const double2* __restrict__ X, int nx, int ny, int nz,
                                                  long long nc, double* __restrict__ partial) {
  __shared__ double scratch[4];
  const int comp = blockIdx.y;
  X += static_cast<long long>(comp) * nc;
  const int nxh = nx / 2 + 1;
  double as = 0.0, ak = 0.0;
  const double two_pi = 6.283185307179586;
  for (long long idx = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x; idx < nc;
       idx += static_cast<long long>(gridDim.x) * 256) {
    const int ix = static_cast<int>(idx % nxh);
    const long long t = idx / nxh;
    const int iy = static_cast<int>(t % ny);
    const int iz = static_cast<int>(t / ny);
    if (ix == 0 && iy == 0 && iz == 0) continue;
    const double w = (ix == 0 || (nx % 2 == 0 && ix == nx / 2)) ? 1.0 : 2.0;
    const double fx = double(ix) / nx;
    const double fy = double(iy <= ny / 2 ? iy : iy - ny) / ny;
    const double fz = double(iz <= nz / 2 ? iz : iz - nz) / nz;
    const double kmag = two_pi * sqrt(fx * fx + fy * fy + fz * fz);
    const double2 c = X[idx];
    const double S = c.x * c.x + c.y * c.y;
    as += w * S;
    ak += w * kmag * S;
  }
  as = block_reduce_d(as, 0, scratch);
  ak = block_reduce_d(ak, 0, scratch);
  if (threadIdx.x == 0) {
    double* out = partial + (static_cast<long long>(comp) * gridDim.x + blockIdx.x) * 2;
    out[0] = as;
    out[1] = ak;
  }
}

// Combine the partial diagnostic records [blocks][3N + 9]: per entry, thread t
// folds blocks t, t + 256, ... in that order, then the workgroup reduces the
// 256 results in a fixed shuffle order, so the result is the same on every
// run.  Entries: N + 3 sums, N maxima, N minima, one maximum, then sums.
__global__ void __launch_bounds__(256) k_reduce_final(const double* __restrict__ partial, double* __restrict__ out,
                                                      int N, int blocks) {
  __shared__ double scratch[4];
  const int rec = reduce_record_len(N);
  const int t = static_cast<int>(threadIdx.x);
  for (int q = 0; q < rec; ++q) {
    const int op = (q < N + 3) ? 0 : (q < 2 * N + 3) ? 1 : (q < 3 * N + 3) ? 2 : (q == 3 * N + 3) ? 1 : 0;
    double acc = op == 0 ? 0.0 : (op == 1 ? -HUGE_VAL : HUGE_VAL);
    for (int b = t; b < blocks; b += 256) {
      const double v = partial[size_t(b) * rec + q];
      acc = op == 0 ? acc + v : (op == 1 ? fmax(acc, v) : fmin(acc, v));
    }
    acc = block_reduce_d(acc, op, scratch);
    if (t == 0) out[q] = acc;
  }
}
#endif

// --------------------------------------------------------------- dispatch
// kernels.hip is compiled once per storage precision (NFLBM_UNIT_STORE = 0, 1,
// 2), each unit instantiating the kernels of that precision, and once more
// (NFLBM_UNIT_STORE = -1) for the reductions and the precision switch.
template <int ST>
using TT = typename StoreT<ST>::T;

// LDS of the update: the concentrations (NE of them; three as a padded
// float record of four) and E_B per position, 1 or 3 planes.
template <int ST>
size_t lds_bytes_for(int lat, int nc, int tx_log2) {
  const int TX = 1 << tx_log2, TY = 256 >> tx_log2;
  const size_t pxy = size_t(TX + 2) * (TY + 2);
  const int npl = lat == 1 ? 3 : 1;
  const int ne = nc - 1;
  const int nep = (sizeof(TT<ST>) == 4 && ne == 3) ? 4 : ne;
  return npl * size_t(nep + 1) * pxy * sizeof(TT<ST>);
}

// LDS of the moment-form reconstruction: one padded record per position.
template <int ST>
size_t conc_m_lds_bytes_for(int lat, int nc, int tx_log2, bool frecord) {
  const int TX = 1 << tx_log2, TY = 256 >> tx_log2;
  const size_t pxy = size_t(TX + 2) * (TY + 2);
  const int npl = 1;   // one plane of records (the z march keeps no other)
  (void)lat;
  const size_t extra = frecord ? 4 : 0;   // (fB, F) of the record form of f
  size_t rec;
  if (sizeof(TT<ST>) == 4) {
    rec = size_t((nc - 1 + 3) / 4 * 4) * 2 + 4 + extra;
    if ((rec * sizeof(TT<ST>) / 16) % 2 == 0) rec += 16 / sizeof(TT<ST>);
  } else {
    rec = size_t(nc - 1) * 2 + 4 + extra;   // field-major, no padding
  }
  return npl * rec * pxy * sizeof(TT<ST>);
}

// The launchers of one (precision, lattice, N), registered by the unit that
// instantiates them (kernels.hip is compiled once per precision, lattice
// and group of N, in parallel) and looked up by the common unit.
struct KernelSet {
  hipError_t (*update)(const StepArgs&, bool, hipStream_t);
  hipError_t (*diag)(const StepArgs&, int, double*, int*, hipStream_t);
  hipError_t (*init)(const InitArgs&, hipStream_t);
  hipError_t (*conc)(const StepArgs&, hipStream_t);
  hipError_t (*batch)(const BatchLaunch&, hipStream_t);
  hipError_t (*expand)(const StepArgs&, hipStream_t);
  hipError_t (*expand_f)(const StepArgs&, void*, hipStream_t);
};
KernelSet& kernel_set(int store, int lat, int nc);

#if defined(NFLBM_UNIT_STORE) && NFLBM_UNIT_STORE >= 0

inline bool any_wall(const StepArgs& a) { return a.wall_x || a.wall_y || a.wall_z || a.bb != nullptr; }
inline bool moments(const StepArgs& a) { return (a.flags & kFlagMoments) != 0; }
// With walls on x only and no solid nodes, a node meets a wall face (in its
// pulls, its stencil or the open-face and outflow rules of that face) only
// at x = 0 and x = nx - 1, in the first and last tile columns; every other
// tile and its one-node halo lie inside the lattice.  The columns between
// them run the periodic variant, whose arithmetic at a node away from walls
// is the wall variant's (pair stencil, pulls in the same order): `inner`
// covers them and `edges` the two edge columns.  False where that does not
// apply (other walls, solids, fewer than three columns, or a launch already
// restricted to some columns).
inline bool split_x_walls(const StepArgs& a, StepArgs& inner, StepArgs& edges) {
  if (!a.wall_x || a.wall_y || a.wall_z || a.bb != nullptr) return false;
  if (a.tiles_x < 3 || a.tile_x0 != 0 || a.tile_xstep != 1) return false;
  inner = a;
  inner.wall_x = 0;      // its tiles and their halos lie strictly inside x
  inner.tile_x0 = 1;
  inner.tiles_x = a.tiles_x - 2;
  edges = a;
  edges.tile_xstep = a.tiles_x - 1;
  edges.tiles_x = 2;
  return true;
}
// storage form of g and f as the update's GM parameter (FP16S keeps its
// binary16 populations of f, so it has no record form)
template <int ST>
inline int storage_gm(const StepArgs& a) {
  if (!moments(a)) return 0;
  return (a.flags & kFlagFRecord) ? 2 : 1;
}

template <class L, int NC, int ST>
hipError_t launch_update_t(const StepArgs& a0, bool fields, hipStream_t s) {
  const auto* P = (const DevParams<TT<ST>>*)(a0.params);
  if (fields) {
    // diagnostics only: one variant (16-wide tiles, walls handled at run time)
    StepArgs a = a0;
    a.tx_log2 = 4;
    a.tiles_x = (a.nx + 15) / 16;
    a.tiles_y = (a.ny + 15) / 16;
    const int blocks = a.tiles_x * a.tiles_y * a.chunks_z;
    const size_t lds = lds_bytes_for<ST>(L::DIM == 3 ? 1 : 0, NC, 4);
    hipLaunchKernelGGL((k_update<L, NC, ST, kModeFields, true, 4, false>), dim3(blocks), dim3(256), lds, s, a, P);
    return hipGetLastError();
  }
  {
    StepArgs inner, edges;
    if (split_x_walls(a0, inner, edges)) {
      hipError_t e = launch_update_t<L, NC, ST>(edges, false, s);
      return e != hipSuccess ? e : launch_update_t<L, NC, ST>(inner, false, s);
    }
  }
  const StepArgs& a = a0;
  const dim3 grid(a.tiles_x * a.tiles_y * a.chunks_z);
  const size_t lds = lds_bytes_for<ST>(L::DIM == 3 ? 1 : 0, NC, a.tx_log2);
#define K_UPD(W, T, G) k_update<L, NC, ST, kModeStep, W, T, G>
#define K_UPD_GM(W, T)                                                                     \
  switch (gm) {                                                                            \
    case 0: hipLaunchKernelGGL((K_UPD(W, T, 0)), grid, dim3(256), lds, s, a, P); break;   \
    case 1: hipLaunchKernelGGL((K_UPD(W, T, 1)), grid, dim3(256), lds, s, a, P); break;   \
    default:                                                                               \
        hipLaunchKernelGGL((K_UPD(W, T, 2)), grid, dim3(256), lds, s, a, P);               \
      break;                                                                               \
  }
  {
    const bool w_ = any_wall(a);
    const int gm = storage_gm<ST>(a);
    if (a.tx_log2 == 6) {
      if (w_) { K_UPD_GM(true, 6) } else { K_UPD_GM(false, 6) }
    } else if (a.tx_log2 == 4) {
      if (w_) { K_UPD_GM(true, 4) } else { K_UPD_GM(false, 4) }
    } else {
      return hipErrorInvalidValue;
    }
  }
#undef K_UPD_GM
#undef K_UPD
  return hipGetLastError();
}

// Diagnostics: the fields mode's launch shape (16-wide tiles, walls handled
// at run time) in reduce mode over at most max_blocks workgroups, then the
// fixed-order sum of their records.
template <class L, int NC, int ST>
hipError_t launch_diag_t(const StepArgs& a0, int max_blocks, double* out, int* nblk, hipStream_t s) {
  const auto* P = (const DevParams<TT<ST>>*)(a0.params);
  StepArgs a = a0;
  a.tx_log2 = 4;
  a.tiles_x = (a.nx + 15) / 16;
  a.tiles_y = (a.ny + 15) / 16;
  const long long tiles = 1LL * a.tiles_x * a.tiles_y * a.chunks_z;
  const int blocks = static_cast<int>(tiles < max_blocks ? tiles : max_blocks);
  const size_t lds = lds_bytes_for<ST>(L::DIM == 3 ? 1 : 0, NC, 4);
  hipLaunchKernelGGL((k_update<L, NC, ST, kModeReduce, true, 4, false>), dim3(blocks), dim3(256), lds, s, a, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  *nblk = blocks;
  return launch_reduce_final(a.diag_partial, out, NC, blocks, s);
}

template <class L, int NC, int ST>
hipError_t launch_init_t(const InitArgs& ia, hipStream_t s) {
  const StepArgs& a = ia.sa;
  const dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4, a.nz);
  const bool w_ = any_wall(a);
  const int gm = storage_gm<ST>(a);
#define K_INIT(W)                                                                                \
  switch (gm) {                                                                                  \
    case 0: hipLaunchKernelGGL((k_init<L, NC, ST, W, 0>), grid, dim3(256), 0, s, ia); break;    \
    case 1: hipLaunchKernelGGL((k_init<L, NC, ST, W, 1>), grid, dim3(256), 0, s, ia); break;    \
    default:                                                                                     \
      hipLaunchKernelGGL((k_init<L, NC, ST, W, 2>), grid, dim3(256), 0, s, ia);                       \
      break;                                                                                     \
  }
  if (w_) { K_INIT(true) } else { K_INIT(false) }
#undef K_INIT
  return hipGetLastError();
}

template <class L, int NC, int ST>
hipError_t launch_conc_t(const StepArgs& a, hipStream_t s) {
  {
    StepArgs inner, edges;
    if (split_x_walls(a, inner, edges)) {
      hipError_t e = launch_conc_t<L, NC, ST>(edges, s);
      return e != hipSuccess ? e : launch_conc_t<L, NC, ST>(inner, s);
    }
  }
  const auto* P = (const DevParams<TT<ST>>*)(a.params);
  const bool w_ = any_wall(a);
  if (moments(a)) {
    const bool fr = storage_gm<ST>(a) == 2;
    const dim3 grid(a.tiles_x * a.tiles_y * a.chunks_z);
    const size_t lds = conc_m_lds_bytes_for<ST>(L::DIM == 3 ? 1 : 0, NC, a.tx_log2, fr);
#define K_CM(W, T, F) k_conc_m<L, NC - 1, ST, W, T, F>
#define K_CM_FR(W, T)                                                                         \
  if (fr) {                                                                                   \
    hipLaunchKernelGGL((K_CM(W, T, true)), grid, dim3(256), lds, s, a, P);                    \
  } else {                                                                                    \
    hipLaunchKernelGGL((K_CM(W, T, false)), grid, dim3(256), lds, s, a, P);                   \
  }
    if (a.tx_log2 == 6) {
      if (w_) { K_CM_FR(true, 6) } else { K_CM_FR(false, 6) }
    } else if (a.tx_log2 == 4) {
      if (w_) { K_CM_FR(true, 4) } else { K_CM_FR(false, 4) }
    } else {
      return hipErrorInvalidValue;
    }
#undef K_CM_FR
#undef K_CM
    return hipGetLastError();
  }
  const int blocks = a.tiles_x * a.tiles_y * a.nz;
  if (w_) hipLaunchKernelGGL((k_conc<L, NC - 1, ST, true>), dim3(blocks), dim3(256), 0, s, a, P);
  else hipLaunchKernelGGL((k_conc<L, NC - 1, ST, false>), dim3(blocks), dim3(256), 0, s, a, P);
  return hipGetLastError();
}

template <class L, int ST>
hipError_t launch_expand_f_t(const StepArgs& a, void* out, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((a.n + 255) / 256);
  if (any_wall(a)) hipLaunchKernelGGL((k_expand_f<L, ST, true>), dim3(blocks), dim3(256), 0, s, a, out);
  else hipLaunchKernelGGL((k_expand_f<L, ST, false>), dim3(blocks), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

template <class L, int NC, int ST>
hipError_t launch_expand_t(const StepArgs& a, hipStream_t s) {
  const auto* P = (const DevParams<TT<ST>>*)(a.params);
  const unsigned blocks = static_cast<unsigned>((a.n + 255) / 256);
  hipLaunchKernelGGL((k_expand_g<L, NC - 1, ST>), dim3(blocks), dim3(256), 0, s, a, P);
  return hipGetLastError();
}

// One time step of every simulation of a batch: the reconstruction over all
// their tiles, then the update over all their tiles.
template <class L, int NC, int ST>
hipError_t launch_batch_t(const BatchLaunch& b, hipStream_t s) {
  const auto* P = static_cast<const DevParams<TT<ST>>*>(b.params);
  const dim3 blk(256);
  const bool fr = b.moments && b.frecord;
  hipError_t e = hipSuccess;
  if (b.phase == 2) {
    // the update only
  } else if (b.moments) {
    const dim3 grid(b.blocks_update);
    const int nb = b.blocks_update;
    const size_t lds = conc_m_lds_bytes_for<ST>(L::DIM == 3 ? 1 : 0, NC, b.tx_log2, fr);
#define K_CMB(W, T, F) k_conc_m_batch<L, NC - 1, ST, W, T, F>
#define K_CMB_FR(W, T)                                                                                \
  if (fr) {                                                                                           \
      hipLaunchKernelGGL((K_CMB(W, T, true)), grid, blk, lds, s, b.args, P, b.work_update, nb);       \
  } else {                                                                                            \
    hipLaunchKernelGGL((K_CMB(W, T, false)), grid, blk, lds, s, b.args, P, b.work_update, nb);        \
  }
    if (b.tx_log2 == 6) {
      if (b.walls) { K_CMB_FR(true, 6) } else { K_CMB_FR(false, 6) }
    } else if (b.tx_log2 == 4) {
      if (b.walls) { K_CMB_FR(true, 4) } else { K_CMB_FR(false, 4) }
    } else {
      return hipErrorInvalidValue;
    }
#undef K_CMB_FR
#undef K_CMB
  } else {
    if (b.walls)
      hipLaunchKernelGGL((k_conc_batch<L, NC - 1, ST, true>), dim3(b.blocks_conc), blk, 0, s, b.args, P, b.work_conc);
    else
      hipLaunchKernelGGL((k_conc_batch<L, NC - 1, ST, false>), dim3(b.blocks_conc), blk, 0, s, b.args, P, b.work_conc);
  }
  e = hipGetLastError();
  if (e != hipSuccess || b.phase == 1) return e;
  const size_t lds = lds_bytes_for<ST>(L::DIM == 3 ? 1 : 0, NC, b.tx_log2);
  const dim3 grid(b.blocks_update);
  const int nb = b.blocks_update;
  const int gm = !b.moments ? 0 : (fr ? 2 : 1);
#define K_UB(W, T, G) k_update_batch<L, NC, ST, W, T, G>
#define K_UB_GM(W, T)                                                                                  \
  switch (gm) {                                                                                        \
    case 0: hipLaunchKernelGGL((K_UB(W, T, 0)), grid, blk, lds, s, b.args, P, b.work_update, nb); break; \
    case 1: hipLaunchKernelGGL((K_UB(W, T, 1)), grid, blk, lds, s, b.args, P, b.work_update, nb); break; \
    default:                                                                                           \
        hipLaunchKernelGGL((K_UB(W, T, 2)), grid, blk, lds, s, b.args, P, b.work_update, nb);          \
      break;                                                                                           \
  }
  if (b.tx_log2 == 6) {
    if (b.walls) { K_UB_GM(true, 6) } else { K_UB_GM(false, 6) }
  } else if (b.tx_log2 == 4) {
    if (b.walls) { K_UB_GM(true, 4) } else { K_UB_GM(false, 4) }
  } else {
    return hipErrorInvalidValue;
  }
#undef K_UB_GM
#undef K_UB
  return hipGetLastError();
}

template <class L, int NC, int ST>
hipError_t diag_launch(const StepArgs& a, int mb, double* out, int* nb, hipStream_t s) {
  return launch_diag_t<L, NC, ST>(a, mb, out, nb, s);
}
template <class L, int NC, int ST>
hipError_t update_launch(const StepArgs& a, bool fields, hipStream_t s) {
  return launch_update_t<L, NC, ST>(a, fields, s);
}

template <class L, int NC>
void register_nc() {
  constexpr int ST = NFLBM_UNIT_STORE;
  KernelSet& k = kernel_set(ST, L::DIM == 3 ? 1 : 0, NC);
  k.update = &update_launch<L, NC, ST>;
  k.diag = &diag_launch<L, NC, ST>;
  k.init = &launch_init_t<L, NC, ST>;
  k.conc = &launch_conc_t<L, NC, ST>;
  k.batch = &launch_batch_t<L, NC, ST>;
  k.expand = &launch_expand_t<L, NC, ST>;
  k.expand_f = &launch_expand_f_t<L, ST>;
}

template <class L, int K>
void register_if_in_unit() {
  if constexpr (NFLBM_UNIT_NC_LO <= K && K <= NFLBM_UNIT_NC_HI) register_nc<L, K>();
}

// This unit's (precision, lattice, range of N): NFLBM_UNIT_LAT 0 = D2Q9,
// 1 = D3Q19; N from NFLBM_UNIT_NC_LO to NFLBM_UNIT_NC_HI.  Registered when
// the library is loaded.
struct UnitRegistrar {
  UnitRegistrar() {
    using L = std::conditional_t<NFLBM_UNIT_LAT == 1, D3Q19, D2Q9>;
    register_if_in_unit<L, 2>();
    register_if_in_unit<L, 3>();
    register_if_in_unit<L, 4>();
    register_if_in_unit<L, 5>();
    register_if_in_unit<L, 6>();
    register_if_in_unit<L, 7>();
    register_if_in_unit<L, 8>();
  }
};
const UnitRegistrar unit_registrar;

#else  // common unit

size_t update_lds_bytes(int lat, int nc, int store, int tx_log2) {
  switch (store) {
    case kStoreF64: return lds_bytes_for<kStoreF64>(lat, nc, tx_log2);
    case kStoreF32: return lds_bytes_for<kStoreF32>(lat, nc, tx_log2);
    default: return lds_bytes_for<kStoreF16S>(lat, nc, tx_log2);
  }
}

size_t conc_m_lds_bytes(int lat, int nc, int store, int tx_log2, bool frecord) {
  switch (store) {
    case kStoreF64: return conc_m_lds_bytes_for<kStoreF64>(lat, nc, tx_log2, frecord);
    case kStoreF32: return conc_m_lds_bytes_for<kStoreF32>(lat, nc, tx_log2, frecord);
    default: return conc_m_lds_bytes_for<kStoreF16S>(lat, nc, tx_log2, frecord);
  }
}

KernelSet& kernel_set(int store, int lat, int nc) {
  static KernelSet table[3][2][kMaxComp + 1] = {};
  return table[store][lat][nc];
}

namespace {
// the registered launchers, or none for an out-of-range request
const KernelSet& kset(int store, int lat, int nc) {
  static const KernelSet none = {};
  if (store < 0 || store > 2 || lat < 0 || lat > 1 || nc < 0 || nc > kMaxComp) return none;
  return kernel_set(store, lat, nc);
}
}  // namespace

hipError_t launch_expand_f(int lat, int store, const StepArgs& a, void* out, hipStream_t s) {
  // the f launcher does not depend on N: any registered N of this lattice
  for (int nc = 2; nc <= kMaxComp; ++nc) {
    const KernelSet& k = kset(store, lat, nc);
    if (k.expand_f) return k.expand_f(a, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_expand(int lat, int nc, int store, const StepArgs& a, hipStream_t s) {
  const KernelSet& k = kset(store, lat, nc);
  return k.expand ? k.expand(a, s) : hipErrorInvalidValue;
}

hipError_t launch_update(int lat, int nc, int store, const StepArgs& a, bool fields, hipStream_t s) {
  const KernelSet& k = kset(store, lat, nc);
  return k.update ? k.update(a, fields, s) : hipErrorInvalidValue;
}

hipError_t launch_diag(int lat, int nc, int store, const StepArgs& a, int max_blocks, double* out, int* blocks,
                       hipStream_t s) {
  const KernelSet& k = kset(store, lat, nc);
  return k.diag ? k.diag(a, max_blocks, out, blocks, s) : hipErrorInvalidValue;
}

hipError_t launch_init(int lat, int nc, int store, const InitArgs& a, hipStream_t s) {
  const KernelSet& k = kset(store, lat, nc);
  return k.init ? k.init(a, s) : hipErrorInvalidValue;
}

hipError_t launch_conc(int lat, int nc, int store, const StepArgs& a, hipStream_t s) {
  const KernelSet& k = kset(store, lat, nc);
  return k.conc ? k.conc(a, s) : hipErrorInvalidValue;
}

hipError_t launch_batch_step(int lat, int nc, int store, const BatchLaunch& b, hipStream_t s) {
  const KernelSet& k = kset(store, lat, nc);
  return k.batch ? k.batch(b, s) : hipErrorInvalidValue;
}

hipError_t launch_build_bb(int lat, const unsigned char* solid, uint32_t* bb, const StepArgs& a,
                           hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((a.n + 255) / 256);
  if (lat == 0) hipLaunchKernelGGL(k_build_bb<D2Q9>, dim3(blocks), dim3(256), 0, s, solid, bb, a);
  else hipLaunchKernelGGL(k_build_bb<D3Q19>, dim3(blocks), dim3(256), 0, s, solid, bb, a);
  return hipGetLastError();
}

hipError_t launch_lambda(const double* C, double* lam, long long total, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  hipLaunchKernelGGL(k_lambda, dim3(blocks), dim3(256), 0, s, C, lam, total);
  return hipGetLastError();
}

hipError_t launch_spectrum(const void* X, int N, int nx, int ny, int nz, long long nc, int blocks,
                           double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_spectrum, dim3(blocks, N), dim3(256), 0, s, static_cast<const double2*>(X), nx, ny, nz, nc,
                     partial);
  return hipGetLastError();
}

hipError_t launch_reduce_final(const double* partial, double* out, int N, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partial, out, N, blocks);
  return hipGetLastError();
}

#endif

}  // namespace nflbm
