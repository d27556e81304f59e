// Reverse-mode (adjoint) kernels of the coupled step, for gradients of the
// time-integrated Poynting flux L = sum_n dt P^n with respect to the eps_r
// and Ms cell maps.  The paper has no adjoint; this is the reverse of the
// forward kernels in kernels.h (same iteration counts, the recorded H-M
// iterates replayed; exact up to rounding, since Step 2's curl term is taken
// back from the two stored E levels), built from:
//   * adj_step_open       opens a reverse step: the stored H levels back into
//                         full-size scratch, and dt dP/dE, dt dP/dH at the
//                         probe plane
//   * adj_mag_prep        per magnetic face: b, d, H_eff^s of the sub-step
//   * adj_mag_iter        reverse of iteration r of the closed-form solve
//                         (N(M), eq:llg_tra4, a = kappa H_eff - d) giving
//                         the cotangent of H_eff per face into Q
//   * adj_gather          transpose of the four-point averages: every face
//                         read by a magnetic face gathers 1/4 of its
//                         readers' Q (fixed order, no atomics)
//   * adj_mag_inv         reverse of b, d, q (eq:llg_tra5/6, eq:iterate_H)
//   * adj_touch,          reverse of the non-magnetic Faraday update: the
//     adj_face_end        face cotangent T splits into the H^s cotangent and
//                         C = -(dt/2 mu0) T for curl E
//   * add_curl_h          E_bar += curl H(C) (transpose of curl E), C read
//                         from the face cotangents as they stand
//   * adj_e_coef          reverse of Step 2 per edge: E_bar <- ca E_bar,
//                         W = cb E_bar, d L / d eps_e accumulated
//   * h_bulk(coef = -1)   H_bar += curl E(W) (transpose of curl H)
//   * copy_gather         the recompute's per-step stores
#pragma once

#include "kernels.h"

namespace mmk {

struct AdjMag {
  const int* idx;
  const unsigned char* nbm;
  const double* Ms;
  const double* kap;
  const double* aoms;
  const double* Ms0[3];   // M^s of the sub-step being reversed
  const double* hlog;     // its iterates H^{(r)}, slot r-1
  double* b[3];
  double* d[3];
  double* hes[3];         // H_eff^s
  double* qb;             // cotangent of q
  double* bb[3];          // cotangent of b
  double* db[3];          // cotangent of d
  double* Mb[3];          // running cotangent of M (of M' on entry, of M^s on exit)
  double* hbit;           // cotangent of the face's own H^{(r)}, r < R
  double* msf_b;          // d L / d Ms_f through N(M)
  double* aoms_b;         // d L / d (alpha/Ms)_f
  int off1, off2, n;
};

__device__ __forceinline__ int adj_family(const AdjMag& a, int t) {
  return t < a.off1 ? 0 : (t < a.off2 ? 1 : 2);
}

// A face of family f at (p[0], p[1], p[2]) counts in the face pass when it
// lies in the grid and is interior along its own axis.
__device__ __forceinline__ bool face_inside(const Geo& g, int f, const int p[3]) {
  return p[0] < g.nx && p[1] < g.ny && p[2] < g.nz && (((g.per >> f) & 1) || p[f] >= 1);
}

// Transpose of x = (b + (a.b) a - a x b) / (1 + |a|^2): cotangents of a, b.
__device__ __forceinline__ void vacus_vjp(const double a[3], const double b[3], const double x[3],
                                          const double xb[3], double ab[3], double bb[3]) {
  const double D = 1.0 + ((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]);
  const double u[3] = {xb[0] / D, xb[1] / D, xb[2] / D};
  const double a_u = (a[0] * u[0] + a[1] * u[1]) + a[2] * u[2];
  const double a_b = (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
  const double x_xb = (x[0] * xb[0] + x[1] * xb[1]) + x[2] * xb[2];
  const double axu[3] = {a[1] * u[2] - a[2] * u[1], a[2] * u[0] - a[0] * u[2], a[0] * u[1] - a[1] * u[0]};
  const double uxb[3] = {u[1] * b[2] - u[2] * b[1], u[2] * b[0] - u[0] * b[2], u[0] * b[1] - u[1] * b[0]};
  for (int c = 0; c < 3; ++c) {
    bb[c] = u[c] + a[c] * a_u + axu[c];
    ab[c] = b[c] * a_u + a_b * u[c] + uxb[c] - 2.0 * a[c] * x_xb / D;
  }
}

// dt dP/dE and dt dP/dH for the node plane x = i0 at node e = j + NY k; the
// level n+1 H of the plane comes from a plane store (see plane_store).
template <typename T>
__device__ __forceinline__ void seed_flux_node(const Geo& g, T* __restrict__ Eby, T* __restrict__ Ebz,
                                               T* __restrict__ Hby, T* __restrict__ Hbz, const T* __restrict__ Ey,
                                               const T* __restrict__ Ez, const T* __restrict__ P, int i0, double w,
                                               int NY, int NZ, int e) {
  const int k = e / NY, j = e - k * NY;
  const int im = dn(i0, g.nx, g.per & 1);
  const long long nn = (long long)NY * NZ;
  if (j < g.ny) {   // + Ey * (Hz(i0-1) + Hz(i0)) / 2
    const int c0 = at(g, i0, j, k), cm = at(g, im, j, k);
    const double hz = 0.5 * (D(P[nn + e]) + D(P[3 * nn + e]));
    const double ey = D(Ey[c0]);
    Eby[c0] = (T)(D(Eby[c0]) + w * hz);
    Hbz[cm] = (T)(D(Hbz[cm]) + w * 0.5 * ey);
    Hbz[c0] = (T)(D(Hbz[c0]) + w * 0.5 * ey);
  }
  if (k < g.nz) {   // - Ez * (Hy(i0-1) + Hy(i0)) / 2
    const int c0 = at(g, i0, j, k), cm = at(g, im, j, k);
    const double hy = 0.5 * (D(P[e]) + D(P[2 * nn + e]));
    const double ez = D(Ez[c0]);
    Ebz[c0] = (T)(D(Ebz[c0]) - w * hy);
    Hby[cm] = (T)(D(Hby[cm]) - w * 0.5 * ez);
    Hby[c0] = (T)(D(Hby[c0]) - w * 0.5 * ez);
  }
}

// b, d and H_eff^s of the sub-step; clears the per-sub-step accumulators.
// With scat_r >= 1 it also puts magnetic iterate scat_r into A (the
// full-size array the next reverse iteration's neighbours read).
template <typename T>
__global__ __launch_bounds__(256) void adj_mag_prep(Geo g, const T* __restrict__ Hs0, const T* __restrict__ Hs1,
                                                   const T* __restrict__ Hs2, AdjMag a, double H0x, double H0y,
                                                   double H0z, T* A0, T* A1, T* A2, int scat_r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const int f = adj_family(a, t);
  const int c = a.idx[t];
  // (and magnetic iterate scat_r into A for the first reverse iteration's neighbours)
  if (scat_r >= 1) (f == 0 ? A0 : (f == 1 ? A1 : A2))[c] = (T)a.hlog[(size_t)(scat_r - 1) * a.n + t];
  int i, j, k;
  face_ijk(g, c, i, j, k);
  HRead<T> Rd;
  Rd.base[0] = Rd.alt[0] = Hs0;
  Rd.base[1] = Rd.alt[1] = Hs1;
  Rd.base[2] = Rd.alt[2] = Hs2;
  Rd.mask = 0;
  const double own = D((f == 0 ? Hs0 : (f == 1 ? Hs1 : Hs2))[c]);
  double he[3];
  h_eff(g, Rd, own, f, i, j, k, H0x, H0y, H0z, he);
  const double kap = a.kap[t], ao = a.aoms[t];
  const double ms[3] = {a.Ms0[0][t], a.Ms0[1][t], a.Ms0[2][t]};
  const double mx = ms[1] * he[2] - ms[2] * he[1];
  const double my = ms[2] * he[0] - ms[0] * he[2];
  const double mz = ms[0] * he[1] - ms[1] * he[0];
  a.b[0][t] = ms[0] + kap * mx;
  a.b[1][t] = ms[1] + kap * my;
  a.b[2][t] = ms[2] + kap * mz;
  for (int q = 0; q < 3; ++q) {
    a.d[q][t] = ao * ms[q];
    a.hes[q][t] = he[q];
    a.bb[q][t] = 0.0;
    a.db[q][t] = 0.0;
  }
  a.qb[t] = 0.0;
}

// Reverse of iteration r on every magnetic face.  Writes the cotangent of
// the face's H_eff (kappa * a_bar) into Q[3 f + c].
template <typename T>
__global__ __launch_bounds__(256) void adj_mag_iter(Geo g, AdjMag a, const T* Hs0, const T* Hs1,
                                                   const T* Hs2, const T* Ho0, const T* Ho1, const T* Ho2,
                                                   const T* A0, const T* A1, const T* A2, T* Hb0, T* Hb1,
                                                   T* Hb2, double* const* Q, int r, int R, double H0x,
                                                   double H0y, double H0z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const int f = adj_family(a, t);
  const int c = a.idx[t];
  int i, j, k;
  face_ijk(g, c, i, j, k);
  double hb, mb[3];
  if (r == R) {
    T* Hb = f == 0 ? Hb0 : (f == 1 ? Hb1 : Hb2);
    hb = D(Hb[c]);
    Hb[c] = (T)0;
    mb[0] = a.Mb[0][t];
    mb[1] = a.Mb[1][t];
    mb[2] = a.Mb[2][t];
  } else {
    hb = a.hbit[t];
    mb[0] = mb[1] = mb[2] = 0.0;
  }
  // H^{(r)} = q - M^{(r)}_f
  a.qb[t] += hb;
  mb[f] -= hb;
  // H_eff^{(r-1)}
  HRead<T> Rd;
  double own;
  if (r == 1) {
    Rd.base[0] = Rd.alt[0] = Hs0;
    Rd.base[1] = Rd.alt[1] = Hs1;
    Rd.base[2] = Rd.alt[2] = Hs2;
    own = D((f == 0 ? Hs0 : (f == 1 ? Hs1 : Hs2))[c]);
  } else {
    Rd.base[0] = Ho0;
    Rd.base[1] = Ho1;
    Rd.base[2] = Ho2;
    Rd.alt[0] = A0;
    Rd.alt[1] = A1;
    Rd.alt[2] = A2;
    own = a.hlog[(size_t)(r - 2) * a.n + t];
  }
  Rd.mask = r == 1 ? 0u : a.nbm[t];
  double he[3];
  h_eff(g, Rd, own, f, i, j, k, H0x, H0y, H0z, he);
  const double kap = a.kap[t], Ms = a.Ms[t];
  const double b[3] = {a.b[0][t], a.b[1][t], a.b[2][t]};
  const double av[3] = {kap * he[0] - a.d[0][t], kap * he[1] - a.d[1][t], kap * he[2] - a.d[2][t]};
  const double ab = (av[0] * b[0] + av[1] * b[1]) + av[2] * b[2];
  const double den = 1.0 + ((av[0] * av[0] + av[1] * av[1]) + av[2] * av[2]);
  const double x[3] = {(b[0] + ab * av[0] - (av[1] * b[2] - av[2] * b[1])) / den,
                       (b[1] + ab * av[1] - (av[2] * b[0] - av[0] * b[2])) / den,
                       (b[2] + ab * av[2] - (av[0] * b[1] - av[1] * b[0])) / den};
  const double nrm = sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]);
  const double xh[3] = {x[0] / nrm, x[1] / nrm, x[2] / nrm};
  const double pr = (xh[0] * mb[0] + xh[1] * mb[1]) + xh[2] * mb[2];
  a.msf_b[t] += pr;
  const double sc = Ms / nrm;
  const double xb[3] = {sc * (mb[0] - xh[0] * pr), sc * (mb[1] - xh[1] * pr), sc * (mb[2] - xh[2] * pr)};
  double abar[3], bbar[3];
  vacus_vjp(av, b, x, xb, abar, bbar);
  for (int q = 0; q < 3; ++q) {
    a.bb[q][t] += bbar[q];
    a.db[q][t] -= abar[q];
    Q[3 * f + q][c] = kap * abar[q];
  }
}

// Transpose of the H_eff reads: for a face u of family cu, the sum of its
// own Q[3cu+cu] and 1/4 of Q[3f+cu] of the four faces of each other family f
// that average it (readers at u + {0, +e_f, -e_cu, +e_f - e_cu}).
// mode 0: iteration r >= 2 (the result is the cotangent of H^{(r-1)}: own
// H iterate of a magnetic face, or the one-shot value of a non-magnetic
// one); mode 1: accumulate into Gb (cotangent of H^s).
template <typename T>
__global__ __launch_bounds__(256) void adj_gather(Geo g, const int* __restrict__ tidx,
                                                 const unsigned char* __restrict__ tfam,
                                                 const int* __restrict__ tmag, int nt, double* const* Q,
                                                 AdjMag a, T* Xb0, T* Xb1, T* Xb2, T* Gb0, T* Gb1, T* Gb2,
                                                 int mode, T* A0, T* A1, T* A2, int scat_r, T* Hb0, T* Hb1,
                                                 T* Hb2, int touch) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  // the next iteration's neighbours: magnetic iterate scat_r into A (the
  // launch covers max(nt, a.n) threads; A is not read here)
  if (scat_r >= 1 && u < a.n) {
    const int ft = adj_family(a, u);
    (ft == 0 ? A0 : (ft == 1 ? A1 : A2))[a.idx[u]] = (T)a.hlog[(size_t)(scat_r - 1) * a.n + u];
  }
  if (u >= nt) return;
  const int cu = tfam[u];
  const int c = tidx[u];
  int p[3];
  face_ijk(g, c, p[0], p[1], p[2]);
  const int n[3] = {g.nx, g.ny, g.nz};
  double s = Q[3 * cu + cu][c];
  double tr = 0.0;
  for (int f = 0; f < 3; ++f) {
    if (f == cu) continue;
    const double* Qf = Q[3 * f + cu];
    const bool pf = (g.per >> f) & 1, pc = (g.per >> cu) & 1;
    // index along f: p[f] (a cell index of u) or p[f]+1; along cu: p[cu] or p[cu]-1
    const int f1 = pf ? (p[f] + 1 == n[f] ? 0 : p[f] + 1) : p[f] + 1;   // <= n_f on a PEC axis: exists
    const bool cm_ok = pc || p[cu] >= 1;
    const int c1 = pc ? (p[cu] == 0 ? n[cu] - 1 : p[cu] - 1) : p[cu] - 1;
    int q[3];
    q[0] = p[0]; q[1] = p[1]; q[2] = p[2];
    double acc = Qf[at(g, q[0], q[1], q[2])];
    q[f] = f1;
    acc += Qf[at(g, q[0], q[1], q[2])];
    if (cm_ok) {
      q[f] = p[f];
      q[cu] = c1;
      acc += Qf[at(g, q[0], q[1], q[2])];
      q[f] = f1;
      acc += Qf[at(g, q[0], q[1], q[2])];
    }
    tr += acc;
  }
  s += 0.25 * tr;
  if (mode == 0) {
    const int m = tmag[u];
    if (m >= 0) {
      a.hbit[m] = s;
    } else {
      T* X = cu == 0 ? Xb0 : (cu == 1 ? Xb1 : Xb2);
      X[c] = (T)(D(X[c]) + s);
    }
  } else {
    T* G = cu == 0 ? Gb0 : (cu == 1 ? Gb1 : Gb2);
    G[c] = (T)(D(G[c]) + s);
  }
  // touch: the face pass's first part on this face (adj_touch mode 0), once
  // X is final (after adj_mag_inv)
  if (touch && face_inside(g, cu, p)) {
    T* H = cu == 0 ? Hb0 : (cu == 1 ? Hb1 : Hb2);
    const T* X = cu == 0 ? Xb0 : (cu == 1 ? Xb1 : Xb2);
    H[c] = (T)(D(H[c]) + D(X[c]));
  }
}

// Reverse of the sub-step invariants q, b, d on every magnetic face.
template <typename T>
__global__ __launch_bounds__(256) void adj_mag_inv(AdjMag a, T* Xb0, T* Xb1, T* Xb2, double* const* Q) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const int f = adj_family(a, t);
  const int c = a.idx[t];
  const double qb = a.qb[t];
  T* X = f == 0 ? Xb0 : (f == 1 ? Xb1 : Xb2);
  X[c] = (T)qb;
  const double kap = a.kap[t], ao = a.aoms[t];
  const double ms[3] = {a.Ms0[0][t], a.Ms0[1][t], a.Ms0[2][t]};
  const double he[3] = {a.hes[0][t], a.hes[1][t], a.hes[2][t]};
  const double bb[3] = {a.bb[0][t], a.bb[1][t], a.bb[2][t]};
  const double db[3] = {a.db[0][t], a.db[1][t], a.db[2][t]};
  // b = M^s + kappa M^s x H_eff^s ; d = (alpha/Ms) M^s ; q = H^s + M^s_f - ...
  const double hxb[3] = {he[1] * bb[2] - he[2] * bb[1], he[2] * bb[0] - he[0] * bb[2],
                         he[0] * bb[1] - he[1] * bb[0]};
  const double bxm[3] = {bb[1] * ms[2] - bb[2] * ms[1], bb[2] * ms[0] - bb[0] * ms[2],
                         bb[0] * ms[1] - bb[1] * ms[0]};
  double mb[3];
  for (int q = 0; q < 3; ++q) {
    mb[q] = bb[q] + kap * hxb[q] + ao * db[q];
    Q[3 * f + q][c] = kap * bxm[q];
  }
  mb[f] += qb;
  a.aoms_b[t] += (db[0] * ms[0] + db[1] * ms[1]) + db[2] * ms[2];
  for (int q = 0; q < 3; ++q) a.Mb[q][t] = mb[q];
}

// The reverse of the non-magnetic Faraday update, per face: T = Hb + Xb is
// the cotangent of the face's Faraday value; the H^s cotangent becomes
// T + Gb and C = -(dt/2 mu0) T feeds curl E.  Wall faces (constant) get 0.
// Xb and Gb are zero off the touched faces, so the pass runs in three
// parts: adj_touch (mode 0, or the last adj_gather with touch) adds Xb on
// the touched faces, add_curl_h reads C straight from Hb, and adj_face_end
// adds Gb there (clearing Xb and Gb) and clears the wall faces.  A face
// counts when it lies in the grid (0 <= i < nx, ...) and is interior along
// its own axis.
template <typename T>
__global__ __launch_bounds__(256) void adj_touch(Geo g, const int* __restrict__ tidx,
                                                const unsigned char* __restrict__ tfam, int nt, T* Hb0, T* Hb1,
                                                T* Hb2, T* Xb0, T* Xb1, T* Xb2, T* Gb0, T* Gb1, T* Gb2, int mode) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nt) return;
  const int f = tfam[u], c = tidx[u];
  T* X = f == 0 ? Xb0 : (f == 1 ? Xb1 : Xb2);
  T* G = f == 0 ? Gb0 : (f == 1 ? Gb1 : Gb2);
  T* H = f == 0 ? Hb0 : (f == 1 ? Hb1 : Hb2);
  int p[3];
  face_ijk(g, c, p[0], p[1], p[2]);
  const bool inside = face_inside(g, f, p);
  if (mode == 0) {
    if (inside) H[c] = (T)(D(H[c]) + D(X[c]));
  } else {
    if (inside) H[c] = (T)(D(H[c]) + D(G[c]));
    X[c] = (T)0;
    G[c] = (T)0;
  }
}

// The face pass's end in one launch: blockIdx.y = f < 3 clears Hb of family
// f on the plane (axis f) = 0 unless the axis is periodic (the wall faces);
// blockIdx.y = 3 is adj_touch mode 1 on the touched faces (interior ones
// only, so the two parts write different faces).
template <typename T>
__global__ __launch_bounds__(256) void adj_face_end(Geo g, const int* __restrict__ tidx,
                                                   const unsigned char* __restrict__ tfam, int nt, T* Hb0, T* Hb1,
                                                   T* Hb2, T* Xb0, T* Xb1, T* Xb2, T* Gb0, T* Gb1, T* Gb2) {
  const int f = blockIdx.y;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f == 3) {
    if (e >= nt) return;
    const int u = (int)e;
    const int fu = tfam[u], c = tidx[u];
    T* X = fu == 0 ? Xb0 : (fu == 1 ? Xb1 : Xb2);
    T* G = fu == 0 ? Gb0 : (fu == 1 ? Gb1 : Gb2);
    T* H = fu == 0 ? Hb0 : (fu == 1 ? Hb1 : Hb2);
    int p[3];
    face_ijk(g, c, p[0], p[1], p[2]);
    if (face_inside(g, fu, p)) H[c] = (T)(D(H[c]) + D(G[c]));
    X[c] = (T)0;
    G[c] = (T)0;
    return;
  }
  if ((g.per >> f) & 1) return;
  const int na = f == 0 ? g.ny : g.nx;   // the plane's first axis (y for f = 0, else x)
  const int nb = f == 2 ? g.ny : g.nz;   // its second (z for f = 0 and 1, y for f = 2)
  if (e >= (long long)na * nb) return;
  const int u = (int)(e % na), v = (int)(e / na);
  if (f == 0) Hb0[at(g, 0, u, v)] = (T)0;
  else if (f == 1) Hb1[at(g, u, 0, v)] = (T)0;
  else Hb2[at(g, u, v, 0)] = (T)0;
}

// E_bar += curl H(C) on interior edges, C = scale * W (W a face field).  Every
// face value an update uses is interior along its own axis.
template <typename T>
__global__ __launch_bounds__(256) void add_curl_h(Geo g, T* __restrict__ Eb0, T* __restrict__ Eb1,
                                                 T* __restrict__ Eb2, const T* __restrict__ W0,
                                                 const T* __restrict__ W1, const T* __restrict__ W2, double scale,
                                                 int kchunk) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(k0 + kchunk, g.nz);
  const bool iin = pxp || i >= 1, jin = pyp || j >= 1;
  const int im = iin ? dn(i, g.nx, pxp) : i;
  const int jm = jin ? dn(j, g.ny, pyp) : j;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  T wx_km = 0, wy_km = 0;
  if (pzp || k0 >= 1) {
    const int km = dn(k0, g.nz, pzp);
    wx_km = (T)(scale * D(W0[at(g, i, j, km)]));
    wy_km = (T)(scale * D(W1[at(g, i, j, km)]));
  }
  for (int k = k0; k < k1; ++k) {
    const bool kin = pzp || k >= 1;
    const int c = at(g, i, j, k);
    const T wx = (T)(scale * D(W0[c])), wy = (T)(scale * D(W1[c])), wz = (T)(scale * D(W2[c]));
    const T wz_jm = (T)(scale * D(W2[at(g, i, jm, k)])), wx_jm = (T)(scale * D(W0[at(g, i, jm, k)]));
    const T wz_im = (T)(scale * D(W2[at(g, im, j, k)])), wy_im = (T)(scale * D(W1[at(g, im, j, k)]));
    if (jin && kin) Eb0[c] = Eb0[c] + (dq(wz - wz_jm, sdy, idy) - dq(wy - wy_km, sdz, idz));
    if (iin && kin) Eb1[c] = Eb1[c] + (dq(wx - wx_km, sdz, idz) - dq(wz - wz_im, sdx, idx));
    if (iin && jin) Eb2[c] = Eb2[c] + (dq(wy - wy_im, sdx, idx) - dq(wx - wx_jm, sdy, idy));
    wx_km = wx;
    wy_km = wy;
  }
}

// Several device-to-device copies in one launch (the per-step state saves of
// the recompute): array blockIdx.y, 8-byte words, grid-stride over x.
constexpr int kCopyMax = 9;
struct CopyBatch {
  const unsigned long long* src[kCopyMax];
  unsigned long long* dst[kCopyMax];
  unsigned long long words[kCopyMax];
};

__global__ __launch_bounds__(256) void copy_batch(CopyBatch b) {
  const int a = blockIdx.y;
  const unsigned long long n = b.words[a];
  const unsigned long long* __restrict__ s = b.src[a];
  unsigned long long* __restrict__ d = b.dst[a];
  for (unsigned long long q = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (unsigned long long)gridDim.x * blockDim.x)
    d[q] = s[q];
}

// The flux seed's H values at level n+1 on the probe plane, per node
// e = j + NY k: Hy(im), Hz(im), Hy(i0), Hz(i0) at out[q * NY * NZ + e] (only
// what the seed reads: Hz where j < ny, Hy where k < nz).  With the capture
// on (fc.buf set, plane p), nodes whose tile is far take the values the far
// tiles' fused pass captured at level n+1 (fmask bits 0 and 1, as the flux
// probe reads them); all others read the fields, which hold level n+1 there.
template <typename T>
struct PlaneStore {
  Geo g;
  const T* Hy;
  const T* Hz;
  FluxCap<T> fc;
  int p;
  const unsigned char* fmask;
  int i0, NY, NZ;
  T* out;   // null: nothing to store
};

template <typename T>
__device__ __forceinline__ void plane_store_node(const PlaneStore<T>& a, int e) {
  const Geo& g = a.g;
  const int NY = a.NY, NZ = a.NZ, i0 = a.i0, p = a.p;
  const FluxCap<T>& fc = a.fc;
  const T* __restrict__ Hy = a.Hy;
  const T* __restrict__ Hz = a.Hz;
  const unsigned char* __restrict__ fmask = a.fmask;
  T* __restrict__ out = a.out;
  const int k = e / NY, j = e - k * NY;
  const int ej = j * NZ + k;   // capture and mask index (z fastest)
  const int im = dn(i0, g.nx, g.per & 1);
  const T* cb = fc.buf ? fc.buf + (long long)p * 6 * fc.nn + ej : nullptr;
  const unsigned m = cb ? (fmask[(long long)p * NY * NZ + ej] & 3u) : 0u;
  const long long nn = (long long)NY * NZ;
  T hym = 0, hzm = 0, hy0 = 0, hz0 = 0;
  if (j < g.ny) {
    hzm = (m & 2u) ? cb[3 * fc.nn] : Hz[at(g, im, j, k)];
    hz0 = (m & 1u) ? cb[5 * fc.nn] : Hz[at(g, i0, j, k)];
  }
  if (k < g.nz) {
    hym = (m & 2u) ? cb[2 * fc.nn] : Hy[at(g, im, j, k)];
    hy0 = (m & 1u) ? cb[4 * fc.nn] : Hy[at(g, i0, j, k)];
  }
  out[e] = hym;
  out[nn + e] = hzm;
  out[2 * nn + e] = hy0;
  out[3 * nn + e] = hz0;
}

template <typename T>
__global__ __launch_bounds__(256) void plane_store(PlaneStore<T> a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < a.NY * a.NZ) plane_store_node(a, e);
}

// The opening of a reverse step in one launch: blockIdx.y = 0 and 1 scatter
// the compact H^n and H^{n+1/2} into their full-size scratch arrays (list
// entries only), blockIdx.y = 2 is the flux seed (seed_flux_node), which
// reads E^{n+1} and the plane store, neither of which the scatters write.
template <typename T>
__global__ __launch_bounds__(256) void adj_step_open(Geo g, const int* __restrict__ gidx,
                                                    const unsigned char* __restrict__ gfam, int ng,
                                                    const T* __restrict__ cn, T* Hn0, T* Hn1, T* Hn2,
                                                    const T* __restrict__ ch, T* Hh0, T* Hh1, T* Hh2, T* Eby,
                                                    T* Ebz, T* Hby, T* Hbz, const T* Ey, const T* Ez,
                                                    const T* __restrict__ P, int i0, double w, int NY, int NZ) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.y < 2) {
    if (e >= ng) return;
    const int f = gfam[e];
    if (blockIdx.y == 0) (f == 0 ? Hn0 : (f == 1 ? Hn1 : Hn2))[gidx[e]] = cn[e];
    else (f == 0 ? Hh0 : (f == 1 ? Hh1 : Hh2))[gidx[e]] = ch[e];
    return;
  }
  if (e >= NY * NZ) return;
  seed_flux_node(g, Eby, Ebz, Hby, Hbz, Ey, Ez, P, i0, w, NY, NZ, e);
}

// Per-step stores of the recompute in one launch: blockIdx.y < ncopy are
// copy_batch's arrays, blockIdx.y = ncopy gathers H at the list entries (when
// ng > 0), the last row stores the previous step's plane values (when ps.out
// is set; the launch comes before anything changes H).
template <typename T>
__global__ __launch_bounds__(256) void copy_gather(CopyBatch b, int ncopy, const int* __restrict__ gidx,
                                                  const unsigned char* __restrict__ gfam, int ng,
                                                  const T* __restrict__ H0, const T* __restrict__ H1,
                                                  const T* __restrict__ H2, T* __restrict__ out, PlaneStore<T> ps) {
  const int a = blockIdx.y;
  if (ps.out && a == (int)gridDim.y - 1) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ps.NY * ps.NZ; e += gridDim.x * blockDim.x)
      plane_store_node(ps, e);
    return;
  }
  if (a < ncopy) {
    const unsigned long long n = b.words[a];
    const unsigned long long* __restrict__ s = b.src[a];
    unsigned long long* __restrict__ d = b.dst[a];
    for (unsigned long long q = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (unsigned long long)gridDim.x * blockDim.x)
      d[q] = s[q];
    return;
  }
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < ng; u += gridDim.x * blockDim.x) {
    const int f = gfam[u];
    out[u] = (f == 0 ? H0 : (f == 1 ? H1 : H2))[gidx[u]];
  }
}

// Reverse of Step 2 on every interior edge: with D = eps/dt + sigma/2,
// ca = (eps/dt - sigma/2)/D, cb = 1/D:  d ca/d eps = (sigma/dt)/D^2,
// d cb/d eps = -(1/dt)/D^2.  epsb accumulates E_bar (E^n d ca + (curl H - J g) d cb);
// W = cb E_bar (to H through curl E), E_bar <- ca E_bar.  The forward set
// E^{n+1} = ca E^n + cb (curl H - J g), so curl H - J g is taken back from
// the two stored E levels as (E^{n+1} - ca E^n) / cb in FP64 (ca and cb are
// the forward's own values, bit for bit; the difference carries the
// forward's rounding, a few ulp of E).  First, the curl transpose of the
// Step 3 reverse that precedes it: E_bar += curl H(C) with C = cscale * Cf
// (the same per-edge expression as add_curl_h).
template <typename T, bool SIG>
__global__ __launch_bounds__(256) void adj_e_coef(Geo g, T* __restrict__ Eb0, T* __restrict__ Eb1,
                                                 T* __restrict__ Eb2, const T* __restrict__ En0,
                                                 const T* __restrict__ En1, const T* __restrict__ En2,
                                                 const T* __restrict__ Ea0, const T* __restrict__ Ea1,
                                                 const T* __restrict__ Ea2, const T* __restrict__ eps,
                                                 const T* __restrict__ sig, T* __restrict__ W0, T* __restrict__ W1,
                                                 T* __restrict__ W2, double* __restrict__ epsb0,
                                                 double* __restrict__ epsb1, double* __restrict__ epsb2, T dt,
                                                 const T* __restrict__ Cf0, const T* __restrict__ Cf1,
                                                 const T* __restrict__ Cf2, double cscale, int kchunk) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(k0 + kchunk, g.nz);
  const bool iin = pxp || i >= 1, jin = pyp || j >= 1;
  const int im = iin ? dn(i, g.nx, pxp) : i;
  const int jm = jin ? dn(j, g.ny, pyp) : j;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  const T e0 = (T)kEps0, half = (T)0.5, quarter = (T)0.25;
  T e_km = 0, e_jm_km = 0, e_im_km = 0, s_km = 0, s_jm_km = 0, s_im_km = 0;
  T wx_km = 0, wy_km = 0;
  if (pzp || k0 >= 1) {
    const int km = dn(k0, g.nz, pzp);
    wx_km = (T)(cscale * D(Cf0[at(g, i, j, km)]));
    wy_km = (T)(cscale * D(Cf1[at(g, i, j, km)]));
    e_km = eps[at(g, i, j, km)];
    e_jm_km = eps[at(g, i, jm, km)];
    e_im_km = eps[at(g, im, j, km)];
    if (SIG) {
      s_km = sig[at(g, i, j, km)];
      s_jm_km = sig[at(g, i, jm, km)];
      s_im_km = sig[at(g, im, j, km)];
    }
  }
  for (int k = k0; k < k1; ++k) {
    const bool kin = pzp || k >= 1;
    const int c = at(g, i, j, k);
    const int cjm = at(g, i, jm, k), cim = at(g, im, j, k);
    const T wx = (T)(cscale * D(Cf0[c])), wy = (T)(cscale * D(Cf1[c])), wz = (T)(cscale * D(Cf2[c]));
    const T wz_jm = (T)(cscale * D(Cf2[cjm])), wx_jm = (T)(cscale * D(Cf0[cjm]));
    const T wz_im = (T)(cscale * D(Cf2[cim])), wy_im = (T)(cscale * D(Cf1[cim]));
    const T e_c = eps[c], e_jm = eps[cjm], e_im = eps[cim], e_imjm = eps[at(g, im, jm, k)];
    T s_c = 0, s_jm = 0, s_im = 0, s_imjm = 0;
    if (SIG) {
      s_c = sig[c];
      s_jm = sig[cjm];
      s_im = sig[cim];
      s_imjm = sig[at(g, im, jm, k)];
    }
    // one edge: given the 4-cell sums and the two E levels, the cotangent
    auto edge = [&](bool in, T esum, T ssum, T en, T e1, T& eb, T& w, double& epsb) {
      if (!in) {
        w = (T)0;
        return;
      }
      const T ee = e0 * (quarter * esum);
      const T a = ee / dt;
      const T sg = SIG ? quarter * ssum : (T)0;
      const T b = sg * half;
      const T den = a + b;
      const T ca = SIG ? (a - b) / den : (T)1;
      const T cb = (T)1 / den;
      const double curl = (D(e1) - D(ca) * D(en)) / D(cb);
      const double d2 = D(den) * D(den);
      const double dca = SIG ? (D(sg) / D(dt)) / d2 : 0.0;
      const double dcb = -(1.0 / D(dt)) / d2;
      const double ebv = D(eb);
      epsb += ebv * (D(en) * dca + curl * dcb);
      w = cb * eb;
      eb = ca * eb;
    };
    {
      T eb = Eb0[c], w;
      if (jin && kin) eb = eb + (dq(wz - wz_jm, sdy, idy) - dq(wy - wy_km, sdz, idz));
      double eps_acc = epsb0[c];
      edge(jin && kin, (e_jm_km + e_km) + (e_jm + e_c), (s_jm_km + s_km) + (s_jm + s_c), En0[c], Ea0[c], eb, w,
           eps_acc);
      Eb0[c] = eb;
      W0[c] = w;
      epsb0[c] = eps_acc;
    }
    {
      T eb = Eb1[c], w;
      if (iin && kin) eb = eb + (dq(wx - wx_km, sdz, idz) - dq(wz - wz_im, sdx, idx));
      double eps_acc = epsb1[c];
      edge(iin && kin, (e_im_km + e_km) + (e_im + e_c), (s_im_km + s_km) + (s_im + s_c), En1[c], Ea1[c], eb, w,
           eps_acc);
      Eb1[c] = eb;
      W1[c] = w;
      epsb1[c] = eps_acc;
    }
    {
      T eb = Eb2[c], w;
      if (iin && jin) eb = eb + (dq(wy - wy_im, sdx, idx) - dq(wx - wx_jm, sdy, idy));
      double eps_acc = epsb2[c];
      edge(iin && jin, (e_imjm + e_jm) + (e_im + e_c), (s_imjm + s_jm) + (s_im + s_c), En2[c], Ea2[c], eb, w,
           eps_acc);
      Eb2[c] = eb;
      W2[c] = w;
      epsb2[c] = eps_acc;
    }
    wx_km = wx;
    wy_km = wy;
    e_km = e_c;
    e_jm_km = e_jm;
    e_im_km = e_im;
    if (SIG) {
      s_km = s_c;
      s_jm_km = s_jm;
      s_im_km = s_im;
    }
  }
}


// d L / d eps_r per cell: the transpose of the 4-cell edge mean, eps0 / 4
// times each edge's cotangent (eb, FP64 on the padded layout), gathered over
// the 12 edges that have the cell among their four -- per component, the
// edges at the cell's two nodes along each transverse axis, skipping PEC
// wall nodes and wrapping periodic ones -- in a fixed order.  Cells of the
// planes k0 <= k < k0 + nk, x fastest, into out.
__global__ __launch_bounds__(256) void adj_eps_cells(Geo g, const double* __restrict__ eb0,
                                                     const double* __restrict__ eb1,
                                                     const double* __restrict__ eb2, int k0, int nk,
                                                     double* __restrict__ out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long plane = (long long)g.nx * g.ny;
  if (q >= plane * nk) return;
  const int i = (int)(q % g.nx);
  const long long r = q / g.nx;
  const int j = (int)(r % g.ny), k = k0 + (int)(r / g.ny);
  const int n[3] = {g.nx, g.ny, g.nz};
  const bool per[3] = {(g.per & 1) != 0, (g.per & 2) != 0, (g.per & 4) != 0};
  const double* eb[3] = {eb0, eb1, eb2};
  double sum = 0.0;
  for (int comp = 0; comp < 3; ++comp) {
    const int t1 = comp == 0 ? 1 : 0, t2 = comp == 2 ? 1 : 2;
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        int p[3] = {i, j, k};
        p[t1] += u;
        p[t2] += v;
        bool interior = true;
        for (int a = 0; a < 3; ++a) {
          if (a == comp) continue;
          if (per[a]) {
            if (p[a] == n[a]) p[a] = 0;
          } else if (p[a] == 0 || p[a] == n[a]) {
            interior = false;
          }
        }
        if (interior) sum += kEps0 * 0.25 * eb[comp][at(g, p[0], p[1], p[2])];
      }
  }
  out[q] = sum;
}

}  // namespace mmk
