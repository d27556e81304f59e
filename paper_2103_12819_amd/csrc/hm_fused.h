// Fused H-M sub-step (Sec. 3.2.2: eq:llg_tra4-6, eq:iterate_H and the
// stopping rule) for grids with many magnetic faces.
//
// The per-iteration launches of kernels.h (hm_pre, hm_step, ...) read the
// iteration-invariant b, d, q and M of every face from HBM at every
// iteration.  Here one launch runs iterations 1..K (K <= 3) of a sub-step
// for a chunk of columns and keeps everything on chip:
//
//   * a chunk is 30 x 6 columns of cells x L planes; its 256 threads cover
//     the chunk plus a one-cell x-y rim (32 x 8 columns), one column each,
//     and march along z (two chunks share a CU, so one's barriers and
//     memory waits overlap the other's arithmetic);
//   * iteration r of a face reads iteration r-1 of its own face and of its
//     eight H_eff neighbours: an x-face reads y- and z-faces at i-1 and i, a
//     y- or z-face reads x-faces at i and i+1 (likewise in y and z), so two
//     iterations back every face of the chunk depends on the chunk plus one
//     cell all round, and one iteration back on a one-sided rim per family.
//     Iteration r is computed on exactly that region (depth K - r), so a
//     one-cell halo in x, y and z serves three iterations;
//   * the iterations form a pipeline along z: at step u the block does
//     iteration 1 on one plane, iteration 2 one plane behind, iteration 3
//     two planes behind; the H iterates go through LDS (a ring of three
//     planes per iteration level); b, q and the last M iterate of a face
//     stay in registers from the plane's first iteration to its last (d is
//     recomputed from M^s, a cache hit);
//   * neighbouring chunks recompute each other's rims (Jacobi iterates are
//     functions of the sub-step's inputs only), so no chunk waits for
//     another; inputs (H^s, M^s) and outputs (H^{(K)}, M^{(K)}) are separate
//     buffers because the rims of the neighbours read the inputs.
//
// Each chunk publishes, for every iteration, the max of |dM|/Ms over the
// faces it owns; hm_more then applies the stopping rule to iterations 1..K.
// When it fires at K the sub-step is done.  Otherwise hm_more recomputes the
// sub-step with the per-face iteration of kernels.h on a co-resident grid
// (a grid barrier per iteration), into the same output buffers: the iterates
// are the same numbers either way, so the result is identical.  K is the
// previous sub-step's count (at most 3), kept on the device, so a recompute
// happens only when the count changes.
//
// The non-magnetic faces of the tiles near magnetic faces take their Faraday
// half step in h_half_db (input buffer -> output buffer) before the fused
// launch; the fused kernel reads those one-shot values from the output
// buffer wherever a magnetic face's H_eff reads a non-magnetic face, and
// overwrites the magnetic faces.
#pragma once

#include "kernels.h"

namespace mmk {

constexpr int kFX = 32, kFY = 8, kFCols = kFX * kFY;  // columns of a chunk, rim included
constexpr int kFIX = kFX - 2;                         // 30 chunk columns in x
constexpr int kFIY = kFY - 2;                         // 6 in y
constexpr int kFMaxK = 3;
constexpr unsigned kNoFace = 0xffffffffu;

template <typename T>
struct FusedArgs {
  const T* Hin[3];        // H^s (the sub-step's input buffer)
  T* Hout[3];             // output buffer; holds the non-magnetic one-shot values
  const T* E[3];
  const double* Min[3];   // M^s (compact, per evolving face)
  double* Mout[3];
  const unsigned* slots;  // per chunk: (L + 2) planes x 3 families x 256 columns, x fastest:
                          // (t << 8) | neighbour mask of evolving face t, or kNoFace
  const int* org;         // per chunk: x0, y0, z0 of the chunk (rim excluded)
  int L;                  // planes per chunk
  int kfix;               // > 0: iterations fixed (parity mode), else K from *kpred
  const int* kpred;       // previous sub-step's count (clamped to 1..3 here)
  Mag m;                  // face constants (fid/ftab or the per-face arrays)
  int nfmat;              // entries of m.ftab (staged in LDS when m.fid is set)
  double H0x, H0y, H0z, hmu0;
  unsigned long long* part;  // part[r * P + chunk], r = 1..K
  int P;
};

struct FaceSt {
  double q, b[3], M[3];   // q of eq:iterate_H, b of eq:llg_tra6, the last M iterate
};
struct PlaneSt {
  FaceSt f[3];
  unsigned s[3];
};

__device__ __forceinline__ int fused_k(const int kfix, const int* kpred) {
  if (kfix > 0) return kfix;
  const int v = *kpred;
  return v < 1 ? 1 : (v > kFMaxK ? kFMaxK : v);
}

// Neighbour q of a face of family F (the numbering of h_eff_load): the H
// component read and its offset in cells.
template <int F>
__device__ __forceinline__ void nb_of(int q, int& comp, int& di, int& dj, int& dk) {
  const int a = q >> 2, w = q & 3;          // transverse component a, slot w
  // slot w: 0 (-n, 0), 1 (0, 0), 2 (-n, +own), 3 (0, +own), where -n steps
  // against the face normal (x-face: -x) and +own along the component's axis
  if (F == 0) {
    comp = a == 0 ? 1 : 2;
    di = (w == 0 || w == 2) ? -1 : 0;
    dj = (a == 0 && w >= 2) ? 1 : 0;
    dk = (a == 1 && w >= 2) ? 1 : 0;
  } else if (F == 1) {
    comp = a == 0 ? 0 : 2;
    dj = (w == 0 || w == 2) ? -1 : 0;
    di = (a == 0 && w >= 2) ? 1 : 0;
    dk = (a == 1 && w >= 2) ? 1 : 0;
  } else {
    comp = a == 0 ? 0 : 1;
    dk = (w == 0 || w == 2) ? -1 : 0;
    di = (a == 0 && w >= 2) ? 1 : 0;
    dj = (a == 1 && w >= 2) ? 1 : 0;
  }
}

__device__ __forceinline__ int ring_at(int lvl, int comp, int slot, int col) {
  return ((lvl * 3 + comp) * 3 + slot) * kFCols + col;
}

__device__ __forceinline__ int slot3(int p) { return (p + 3) % 3; }

// Where iteration r of family F is computed, at depth dep = K - r below the
// last iteration: in the chunk's own columns (dep 0), on the one-sided rim
// its neighbours read (dep 1), on the whole rim (dep 2); ex, ey are the
// column in the 32 x 8 block (chunk columns 1..30 x 1..6) and p the plane
// (chunk planes 0..L-1).
__device__ __forceinline__ bool in_region(int dep, int F, int ex, int ey, int p, int L) {
  if (dep == 0) return ex >= 1 && ex < kFX - 1 && ey >= 1 && ey < kFY - 1 && p >= 0 && p < L;
  if (dep == 1) {
    if (F == 0) return ex >= 1 && ey < kFY - 1 && p >= -1 && p < L;
    if (F == 1) return ex < kFX - 1 && ey >= 1 && p >= -1 && p < L;
    return ex < kFX - 1 && ey < kFY - 1 && p >= 0 && p < L + 1;
  }
  return p >= -1 && p < L + 1;
}

// Index offsets of the neighbours of this thread's column (i -/+ 1, j -/+ 1
// in the padded layout), wrapped on periodic axes.
struct FusedOff {
  int xm, xp, ym, yp;
};

__device__ __forceinline__ void face_consts_lds(const Mag& m, const double* tab, int t, double& Ms, double& kap,
                                                double& aoms) {
  if (m.fid) {
    const double* e = tab + 3 * (int)m.fid[t];
    Ms = e[0];
    kap = e[1];
    aoms = e[2];
  } else {
    Ms = m.Ms[t];
    kap = m.kap[t];
    aoms = m.aoms[t];
  }
}

// max over the three components of |dM_c| / Ms as residual bits: the max
// of |dM_c| taken on the bit patterns (a NaN wins), then one division (the
// quotient by Ms > 0 is monotone, so this equals the max of the three
// quotients).
__device__ __forceinline__ unsigned long long resid3(const double mn[3], const double mo[3], double Ms) {
  unsigned long long u = rbits(mn[0] - mo[0]);
  const unsigned long long u1 = rbits(mn[1] - mo[1]), u2 = rbits(mn[2] - mo[2]);
  u = u1 > u ? u1 : u;
  u = u2 > u ? u2 : u;
  return rbits(__longlong_as_double((long long)u) / Ms);
}

// Iteration 1 of evolving face t of family F at (i, j, k): the invariants
// b and q of eq:llg_tra6 / eq:iterate_H from H^s, M^s and curl E, then the
// solve (the arithmetic of hm_pre, so the results agree to the bit).
// Both take `act`: an inactive face (none here, or outside the iteration's
// region) runs the same code on index 0 of every array (always in range)
// and its results are dropped, so the three families' loads can all be
// issued together.
template <typename T, int F>
__device__ __forceinline__ void fused_first(const Geo& g, const FusedArgs<T>& a, const double* tab, unsigned s,
                                            bool act, int c, FusedOff o, int ozm, int ozp, FaceSt& st, T& hv,
                                            unsigned long long& rb, bool count) {
  const int t = act ? (int)(s >> 8) : 0;
  if (!act) {
    c = 0;
    o.xm = o.xp = o.ym = o.yp = 0;
    ozm = ozp = 0;
  }
  double Ms, kap, aoms;
  face_consts_lds(a.m, tab, t, Ms, kap, aoms);
  const double ms[3] = {a.Min[0][t], a.Min[1][t], a.Min[2][t]};
  // curl E at the face (reference operation order, FP64 divisions)
  double Cf;
  if (F == 0)
    Cf = (D(a.E[2][c + o.yp]) - D(a.E[2][c])) / g.dy - (D(a.E[1][c + ozp]) - D(a.E[1][c])) / g.dz;
  else if (F == 1)
    Cf = (D(a.E[0][c + ozp]) - D(a.E[0][c])) / g.dz - (D(a.E[2][c + o.xp]) - D(a.E[2][c])) / g.dx;
  else
    Cf = (D(a.E[1][c + o.xp]) - D(a.E[1][c])) / g.dx - (D(a.E[0][c + o.yp]) - D(a.E[0][c])) / g.dy;
  double nv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int comp, di, dj, dk;
    nb_of<F>(q, comp, di, dj, dk);
    const int off = (di < 0 ? o.xm : (di > 0 ? o.xp : 0)) + (dj < 0 ? o.ym : (dj > 0 ? o.yp : 0)) +
                    (dk < 0 ? ozm : (dk > 0 ? ozp : 0));
    nv[q] = D(a.Hin[comp][c + off]);
  }
  const double hs = D(a.Hin[F][c]);
  double he[3];
  h_eff_sum(nv, hs, F, a.H0x, a.H0y, a.H0z, he);
  const double mx = ms[1] * he[2] - ms[2] * he[1];
  const double my = ms[2] * he[0] - ms[0] * he[2];
  const double mz = ms[0] * he[1] - ms[1] * he[0];
  st.q = hs + ms[F] - a.hmu0 * Cf;
  st.b[0] = ms[0] + kap * mx;
  st.b[1] = ms[1] + kap * my;
  st.b[2] = ms[2] + kap * mz;
  const double d[3] = {aoms * ms[0], aoms * ms[1], aoms * ms[2]};
  double mn[3];
  llg_solve(he, kap, d, st.b, Ms, mn);
  hv = (T)(st.q - mn[F]);
  if (count && act) {
    const unsigned long long bb = resid3(mn, ms, Ms);
    rb = bb > rb ? bb : rb;
  }
  st.M[0] = mn[0];
  st.M[1] = mn[1];
  st.M[2] = mn[2];
}

// Iteration r >= 2 of the same face: H^{(r-1)} of the evolving neighbours
// from the ring (level lvl = r - 2), of the other neighbours from Hout (the
// arithmetic of iterate_faces).
template <typename T, int F>
__device__ __forceinline__ void fused_next(const FusedArgs<T>& a, const double* tab, const T* ring, int lvl,
                                           unsigned s, bool act, int c, FusedOff o, int ozm, int ozp, int col,
                                           int p, FaceSt& st, T& hv, unsigned long long& rb, bool count) {
  const int t = act ? (int)(s >> 8) : 0;
  const unsigned mask = act ? (s & 255u) : 0u;
  if (!act) {
    c = 0;
    o.xm = o.xp = o.ym = o.yp = 0;
    ozm = ozp = 0;
  }
  double Ms, kap, aoms;
  face_consts_lds(a.m, tab, t, Ms, kap, aoms);
  const double d[3] = {aoms * a.Min[0][t], aoms * a.Min[1][t], aoms * a.Min[2][t]};
  double nv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int comp, di, dj, dk;
    nb_of<F>(q, comp, di, dj, dk);
    if ((mask >> q) & 1u) {
      nv[q] = D(ring[ring_at(lvl, comp, slot3(p + dk), col + di + kFX * dj)]);   // in range: see in_region
    } else {
      const int off = (di < 0 ? o.xm : (di > 0 ? o.xp : 0)) + (dj < 0 ? o.ym : (dj > 0 ? o.yp : 0)) +
                      (dk < 0 ? ozm : (dk > 0 ? ozp : 0));
      nv[q] = D(a.Hout[comp][c + off]);
    }
  }
  const double own = D(ring[ring_at(lvl, F, slot3(p), act ? col : 0)]);
  double he[3];
  h_eff_sum(nv, own, F, a.H0x, a.H0y, a.H0z, he);
  double mn[3];
  llg_solve(he, kap, d, st.b, Ms, mn);
  hv = (T)(st.q - mn[F]);
  if (count && act) {
    const unsigned long long bb = resid3(mn, st.M, Ms);
    rb = bb > rb ? bb : rb;
  }
  st.M[0] = mn[0];
  st.M[1] = mn[1];
  st.M[2] = mn[2];
}

template <typename T>
__device__ __forceinline__ void fused_out(const FusedArgs<T>& a, int F, int c, unsigned s, const FaceSt& st,
                                          T hv) {
  const int t = (int)(s >> 8);
  a.Hout[F][c] = hv;
  a.Mout[0][t] = st.M[0];
  a.Mout[1][t] = st.M[1];
  a.Mout[2][t] = st.M[2];
}

struct FusedCol {
  int ex, ey, col;  // column in the block
  int cij;          // padded index of (i, j, 0)
  FusedOff o;
  bool own;         // a chunk column inside the grid: this chunk writes its faces
  int z0, L, K;
};

// One pipeline step u: iteration 1 on plane p1 = u - (K > 1) into Nw,
// iteration 2 one plane behind on Md, iteration 3 two planes behind on Od.
// pf holds the slots of plane p1 (loaded one step ahead) and is refilled
// with those of the next plane.
template <typename T>
__device__ __forceinline__ void fused_step(const Geo& g, const FusedArgs<T>& a, T* ring, const double* tab,
                                           const unsigned* sl, const FusedCol& C, int u, PlaneSt& Nw,
                                           PlaneSt& Md, PlaneSt& Od, unsigned (&pf)[3],
                                           unsigned long long rb[3]) {
  const bool pzp = g.per & 4;
  const int K = C.K;
  // the plane's padded offset and its z neighbours' offsets
  auto plane = [&](int p, int& c, int& ozm, int& ozp) {
    int k = C.z0 + p;
    if (pzp) k = (k % g.nz + g.nz) % g.nz;
    c = C.cij + g.sz * k;
    ozm = (pzp && k == 0) ? g.sz * (g.nz - 1) : -g.sz;
    ozp = (pzp && k == g.nz - 1) ? -g.sz * (g.nz - 1) : g.sz;
  };
  // faces this chunk writes and counts: chunk columns and planes inside the
  // grid (on a periodic axis the overhang past the end is rim)
  auto owned = [&](int p) { return C.own && p >= 0 && p < C.L && C.z0 + p < g.nz; };
  // iteration 1
  const int p1 = u - (K > 1 ? 1 : 0);
  {
    bool act[3];
#pragma unroll
    for (int F = 0; F < 3; ++F) {
      Nw.s[F] = pf[F];
      act[F] = pf[F] != kNoFace && in_region(K - 1, F, C.ex, C.ey, p1, C.L);
      if (!act[F]) Nw.s[F] = kNoFace;
    }
    if (p1 + 2 < C.L + 2) {
      const unsigned* row = sl + (size_t)(p1 + 2) * 3 * kFCols + C.col;
      pf[0] = row[0];
      pf[1] = row[kFCols];
      pf[2] = row[2 * kFCols];
    } else {
      pf[0] = pf[1] = pf[2] = kNoFace;
    }
    if (act[0] || act[1] || act[2]) {
      int c, ozm, ozp;
      plane(p1, c, ozm, ozp);
      const bool cnt = owned(p1);
#pragma unroll
      for (int F = 0; F < 3; ++F) {
        if (!act[F]) continue;
        T hv;
        if (F == 0) fused_first<T, 0>(g, a, tab, Nw.s[0], true, c, C.o, ozm, ozp, Nw.f[0], hv, rb[0], cnt);
        else if (F == 1) fused_first<T, 1>(g, a, tab, Nw.s[1], true, c, C.o, ozm, ozp, Nw.f[1], hv, rb[0], cnt);
        else fused_first<T, 2>(g, a, tab, Nw.s[2], true, c, C.o, ozm, ozp, Nw.f[2], hv, rb[0], cnt);
        if (K == 1) {
          if (cnt) fused_out(a, F, c, Nw.s[F], Nw.f[F], hv);
        } else {
          ring[ring_at(0, F, slot3(p1), C.col)] = hv;
        }
      }
    }
  }
  if (K < 2) return;
  __syncthreads();
  // iteration 2
  const int p2 = p1 - 1;
  {
    bool act[3];
#pragma unroll
    for (int F = 0; F < 3; ++F) {
      act[F] = Md.s[F] != kNoFace && in_region(K - 2, F, C.ex, C.ey, p2, C.L);
      if (!act[F]) Md.s[F] = kNoFace;
    }
    if (act[0] || act[1] || act[2]) {
      int c, ozm, ozp;
      plane(p2, c, ozm, ozp);
      const bool cnt = owned(p2);
#pragma unroll
      for (int F = 0; F < 3; ++F) {
        if (!act[F]) continue;
        T hv;
        if (F == 0) fused_next<T, 0>(a, tab, ring, 0, Md.s[0], true, c, C.o, ozm, ozp, C.col, p2, Md.f[0], hv, rb[1], cnt);
        else if (F == 1) fused_next<T, 1>(a, tab, ring, 0, Md.s[1], true, c, C.o, ozm, ozp, C.col, p2, Md.f[1], hv, rb[1], cnt);
        else fused_next<T, 2>(a, tab, ring, 0, Md.s[2], true, c, C.o, ozm, ozp, C.col, p2, Md.f[2], hv, rb[1], cnt);
        if (K == 2) {
          if (cnt) fused_out(a, F, c, Md.s[F], Md.f[F], hv);
        } else {
          ring[ring_at(1, F, slot3(p2), C.col)] = hv;
        }
      }
    }
  }
  __syncthreads();
  if (K < 3) return;
  // iteration 3
  const int p3 = p2 - 1;
  if (owned(p3)) {
    bool act[3];
#pragma unroll
    for (int F = 0; F < 3; ++F) act[F] = Od.s[F] != kNoFace;
    if (act[0] || act[1] || act[2]) {
      int c, ozm, ozp;
      plane(p3, c, ozm, ozp);
#pragma unroll
      for (int F = 0; F < 3; ++F) {
        if (!act[F]) continue;
        T hv;
        if (F == 0) fused_next<T, 0>(a, tab, ring, 1, Od.s[0], true, c, C.o, ozm, ozp, C.col, p3, Od.f[0], hv, rb[2], true);
        else if (F == 1) fused_next<T, 1>(a, tab, ring, 1, Od.s[1], true, c, C.o, ozm, ozp, C.col, p3, Od.f[1], hv, rb[2], true);
        else fused_next<T, 2>(a, tab, ring, 1, Od.s[2], true, c, C.o, ozm, ozp, C.col, p3, Od.f[2], hv, rb[2], true);
        fused_out(a, F, c, Od.s[F], Od.f[F], hv);
      }
    }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kFCols) void hm_fused(Geo g, FusedArgs<T> a) {
  __shared__ T ring[2 * 3 * 3 * kFCols];
  __shared__ double tab[3 * 256];
  const int tid = threadIdx.x;
  if (a.m.fid)
    for (int q = tid; q < 3 * a.nfmat; q += kFCols) tab[q] = a.m.ftab[q];
  FusedCol C;
  C.ex = tid % kFX;
  C.ey = tid / kFX;
  C.col = tid;
  const int qc = blockIdx.x;
  C.z0 = a.org[3 * qc + 2];
  C.L = a.L;
  C.K = fused_k(a.kfix, a.kpred);
  const bool pxp = g.per & 1, pyp = g.per & 2;
  int i = a.org[3 * qc] - 1 + C.ex, j = a.org[3 * qc + 1] - 1 + C.ey;
  const bool in_grid = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
  // wrap on periodic axes; elsewhere a column off the grid has no faces (its
  // slots say so) and its indices are never used
  if (pxp) i = (i % g.nx + g.nx) % g.nx;
  if (pyp) j = (j % g.ny + g.ny) % g.ny;
  C.cij = i + g.px * j;
  C.o.xm = (pxp && i == 0) ? g.nx - 1 : -1;
  C.o.xp = (pxp && i == g.nx - 1) ? -(g.nx - 1) : 1;
  C.o.ym = (pyp && j == 0) ? g.px * (g.ny - 1) : -g.px;
  C.o.yp = (pyp && j == g.ny - 1) ? -g.px * (g.ny - 1) : g.px;
  C.own = in_grid && C.ex >= 1 && C.ex < kFX - 1 && C.ey >= 1 && C.ey < kFY - 1;
  const unsigned* sl = a.slots + (size_t)qc * (a.L + 2) * 3 * kFCols;
  PlaneSt S0, S1, S2;
  for (int F = 0; F < 3; ++F) S0.s[F] = S1.s[F] = S2.s[F] = kNoFace;
  unsigned long long rb[3] = {0ull, 0ull, 0ull};
  // slots of the first plane of iteration 1 (p = -1 when K > 1, else 0)
  unsigned pf[3];
  {
    const unsigned* row = sl + (size_t)(C.K > 1 ? 0 : 1) * 3 * kFCols + C.col;
    pf[0] = row[0];
    pf[1] = row[kFCols];
    pf[2] = row[2 * kFCols];
  }
  __syncthreads();
  const int NS = a.L + C.K - 1 + (C.K > 1 ? 1 : 0);
  for (int u = 0; u < NS; u += 3) {
    fused_step(g, a, ring, tab, sl, C, u, S0, S1, S2, pf, rb);
    if (u + 1 < NS) fused_step(g, a, ring, tab, sl, C, u + 1, S2, S0, S1, pf, rb);
    if (u + 2 < NS) fused_step(g, a, ring, tab, sl, C, u + 2, S1, S2, S0, pf, rb);
  }
  for (int r = 1; r <= C.K; ++r) {
    const unsigned long long v = block_max_u64(rb[r - 1]);
    if (tid == 0)
      __hip_atomic_store(&a.part[(size_t)r * a.P + qc], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// The Faraday half step of the near tiles from the input buffer into the
// output buffer (the arithmetic of h_bulk with NP = 1, so every face gets
// the value h_bulk would store; the magnetic faces are overwritten later).
// ---------------------------------------------------------------------------
template <typename T, bool MU>
__global__ __launch_bounds__(256) void h_half_db(Geo g, const T* __restrict__ Hxi, const T* __restrict__ Hyi,
                                                const T* __restrict__ Hzi, T* __restrict__ Hxo,
                                                T* __restrict__ Hyo, T* __restrict__ Hzo,
                                                const T* __restrict__ Ex, const T* __restrict__ Ey,
                                                const T* __restrict__ Ez, const T* __restrict__ mu, T coef0, T h,
                                                Tiles tl, FluxCap<T> cap = {}) {
  int i, j, k0, k1;
  tile_span(tl, g.nz, i, j, k0, k1);
  const int tx = i;
  i += threadIdx.x;
  j += threadIdx.y;
  // flux-plane capture of the near tiles' plane nodes at level n+1 (the
  // last half step of a step; see CapRole)
  __shared__ T stash[4 * 6 * kCapPlanesZ];
  const CapRole cr = cap_role(cap, tx, j, k0);
  if (j >= g.ny || k0 >= k1) return;
  const bool capw = cr.l0 >= 0 || cr.lm >= 0;   // wave-uniform
  T* st = stash + __builtin_amdgcn_readfirstlane(threadIdx.y) * 6 * kCapPlanesZ;
  if (i < g.nx) {
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const bool iin = pxp || i >= 1;
  const bool jin = pyp || j >= 1;
  const int ip = up(i, g.nx, pxp), jp = up(j, g.ny, pyp);
  const int im = iin ? dn(i, g.nx, pxp) : i;
  const int jm = jin ? dn(j, g.ny, pyp) : j;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  const T mu0 = (T)kMu0, half = (T)0.5;
  T ex_k = Ex[at(g, i, j, k0)];
  T ey_k = Ey[at(g, i, j, k0)];
  T mu_km = 0;
  if (MU && (pzp || k0 >= 1)) mu_km = mu[at(g, i, j, dn(k0, g.nz, pzp))];
  for (int k = k0; k < k1; ++k) {
    const int kp = up(k, g.nz, pzp);
    const int c = at(g, i, j, k);
    const T ex_kp = Ex[at(g, i, j, kp)], ey_kp = Ey[at(g, i, j, kp)];
    const T ez = Ez[c], ez_jp = Ez[at(g, i, jp, k)], ez_ip = Ez[at(g, ip, j, k)];
    const T ey_ip = Ey[at(g, ip, j, k)], ex_jp = Ex[at(g, i, jp, k)];
    T mu_c = 0, mu_im = 0, mu_jm = 0;
    if (MU) {
      mu_c = mu[c];
      mu_im = mu[at(g, im, j, k)];
      mu_jm = mu[at(g, i, jm, k)];
    }
    if (iin) {
      const T curl = dq(ez_jp - ez, sdy, idy) - dq(ey_kp - ey_k, sdz, idz);
      const T cf = MU ? h / (mu0 * (half * (mu_im + mu_c))) : coef0;
      Hxo[c] = Hxi[c] - cf * curl;
    }
    T hy1 = Hyi[c], hz1 = Hzi[c];
    if (jin) {
      const T curl = dq(ex_kp - ex_k, sdz, idz) - dq(ez_ip - ez, sdx, idx);
      const T cf = MU ? h / (mu0 * (half * (mu_jm + mu_c))) : coef0;
      hy1 = hy1 - cf * curl;
      Hyo[c] = hy1;
    }
    if (pzp || k >= 1) {
      const T curl = dq(ey_ip - ey_k, sdx, idx) - dq(ex_jp - ex_k, sdy, idy);
      const T cf = MU ? h / (mu0 * (half * (mu_km + mu_c))) : coef0;
      hz1 = hz1 - cf * curl;
      Hzo[c] = hz1;
    }
    if (capw) cap_park(cr, st, k - k0, ey_k, ez, hy1, hz1);
    ex_k = ex_kp;
    ey_k = ey_kp;
    if (MU) mu_km = mu_c;
  }
  }
  if (capw) cap_flush(cr, cap, st, k1 - k0);
}

// Copy H (three components) on the cells of the listed tiles.
template <typename T>
__global__ __launch_bounds__(256) void copy_tiles(Geo g, const T* __restrict__ s0, const T* __restrict__ s1,
                                                 const T* __restrict__ s2, T* __restrict__ d0,
                                                 T* __restrict__ d1, T* __restrict__ d2, Tiles tl) {
  int i, j, k0, k1;
  tile_span(tl, g.nz, i, j, k0, k1);
  i += threadIdx.x;
  j += threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  for (int k = k0; k < k1; ++k) {
    const int c = at(g, i, j, k);
    d0[c] = s0[c];
    d1[c] = s1[c];
    d2[c] = s2[c];
  }
}

// ---------------------------------------------------------------------------
// After hm_fused: the stopping rule on iterations 1..K.  Done when it fires
// at K (the common case: every block returns after reading the partials).
// Otherwise the whole sub-step is recomputed here from its inputs with the
// per-face iteration (iteration 1 as hm_pre, r >= 2 as hm_step) on this
// co-resident grid, one grid barrier per iteration, H iterates alternating
// between S (odd r) and Hout (even r), M updated in Mout.
// ---------------------------------------------------------------------------
template <typename T>
struct MoreArgs {
  const T* Hin[3];
  T* Hout[3];
  T* S[3];                 // shadow for the odd iterates
  const T* E[3];
  const double* Min[3];
  Mag m;                   // m.M = Mout; b, d, q scratch arrays
  double H0x, H0y, H0z, hmu0;
  const unsigned long long* fpart;   // hm_fused's partials (P_f per iteration)
  int Pf;
  int kfix;
  int* kpred;
};

template <typename T>
__global__ __launch_bounds__(256) void hm_more(Geo g, MoreArgs<T> a, Ctl C, int* iters_out, int* ring,
                                              unsigned int* bar, int* err) {
  const int K = fused_k(a.kfix, a.kpred);
  // residuals of iterations 1..K from the fused launch
  int rstop = 0;
  bool bad = false;
  unsigned long long bits = 0;
  for (int r = 1; r <= K && !rstop; ++r) {
    unsigned long long v = 0;
    const unsigned long long* p = a.fpart + (size_t)r * a.Pf;
    for (int q = threadIdx.x; q < a.Pf; q += blockDim.x) {
      const unsigned long long w = load_u64(&p[q]);
      v = w > v ? w : v;
    }
    v = block_max_u64(v);
    if (stop_rule(C, r, v, bad)) {
      rstop = r;
      bits = v;
    }
  }
  int rfin;
  if (rstop == K) {
    rfin = K;
  } else {
    // recompute from the inputs on this grid
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    const Mag& m = a.m;
    unsigned long long rb = 0;
    for (int t = tid; t < m.n; t += nth) {
      const int f = face_family(m, t);
      const int c = m.idx[t];
      double Ms, kap, aoms;
      face_consts(m, t, Ms, kap, aoms);
      const double ms[3] = {a.Min[0][t], a.Min[1][t], a.Min[2][t]};
      int i, j, k;
      face_ijk(g, c, i, j, k);
      Fields<T> FE;
      for (int q = 0; q < 3; ++q) {
        FE.E[q] = (T*)a.E[q];
        FE.H[q] = FE.A[q] = FE.B[q] = nullptr;
      }
      const double Cf = curl_e_face(g, FE, f, i, j, k);
      HRead<T> Rd;
      for (int q = 0; q < 3; ++q) Rd.base[q] = Rd.alt[q] = a.Hin[q];
      Rd.mask = 0;
      const double hs = D(a.Hin[f][c]);
      double nv[8];
      h_eff_load(g, Rd, f, i, j, k, nv);
      double he[3];
      h_eff_sum(nv, hs, f, a.H0x, a.H0y, a.H0z, he);
      const double mx = ms[1] * he[2] - ms[2] * he[1];
      const double my = ms[2] * he[0] - ms[0] * he[2];
      const double mz = ms[0] * he[1] - ms[1] * he[0];
      const double q = hs + ms[f] - a.hmu0 * Cf;
      const double b[3] = {ms[0] + kap * mx, ms[1] + kap * my, ms[2] + kap * mz};
      const double d[3] = {aoms * ms[0], aoms * ms[1], aoms * ms[2]};
      double mn[3];
      llg_solve(he, kap, d, b, Ms, mn);
      for (int q3 = 0; q3 < 3; ++q3) {
        m.b[q3][t] = b[q3];
        m.d[q3][t] = d[q3];
        const unsigned long long bb = rbits(fabs(mn[q3] - ms[q3]) / Ms);
        rb = bb > rb ? bb : rb;
        m.M[q3][t] = mn[q3];
      }
      m.q[t] = q;
      tri(a.S)(f)[c] = (T)(q - mn[f]);
    }
    publish_residual(C, 1, rb);
    int r = 2;
    if (!grid_barrier(bar)) {
      if (threadIdx.x == 0) atomicOr(err, 4);
    } else {
      Fields<T> F;
      for (int q = 0; q < 3; ++q) {
        F.E[q] = (T*)a.E[q];
        F.H[q] = a.Hout[q];
        F.A[q] = F.B[q] = nullptr;
      }
      for (;;) {
        if (stop_rule(C, r - 1, residual_bits(C, r - 1), bad)) break;
        const Tri<T> prev = (r - 1) & 1 ? tri(a.S) : tri(a.Hout);
        const Tri<T> out = r & 1 ? tri(a.S) : tri(a.Hout);
        const unsigned long long lb = iterate_faces(g, m, F, prev, out, tid, nth, a.H0x, a.H0y, a.H0z, r, err);
        publish_residual(C, r, lb);
        if (!grid_barrier(bar)) {
          if (threadIdx.x == 0) atomicOr(err, 4);
          r += 1;
          break;
        }
        ++r;
      }
    }
    rfin = r - 1;
    bits = residual_bits(C, rfin);
    // an odd final count left the magnetic faces' H in S
    if (rfin & 1)
      for (int t = tid; t < m.n; t += nth) {
        const int f = face_family(m, t);
        const int c = m.idx[t];
        tri(a.Hout)(f)[c] = tri(a.S)(f)[c];
      }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    iters_out[0] = rfin;
    ring[0] = rfin;
    *a.kpred = rfin;
    bool b2;
    stop_rule(C, rfin, bits, b2);
    int e = 0;
    if (b2) e |= 2;
    else if (C.fixed_iter <= 0) {
      const double rv = __longlong_as_double((long long)bits);
      if (!(rv < C.tol)) e |= 1;
    }
    if (e) atomicOr(err, e);
  }
}

}  // namespace mmk
