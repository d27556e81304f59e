// Device kernels of the coupled Maxwell-LLG step for gfx950 (CDNA4).
//
// Scheme: Yao, Jambunathan, Zeng & Nonaka, Sec. 3.2.2 (second-order coupled
// scheme) on the Yee grid of Sec. 3.1.  One step is
//   Step 1: H-M sub-step with curl E^n     (hm_pre -> h_bulk -> hm_iter)
//   Step 2: E update with the soft source   (e_update)
//   Step 3: H-M sub-step with curl E^{n+1} (hm_pre -> h_bulk -> hm_iter)
//   probes at level n+1                     (probe_points, probe_flux)
//
// Storage: every field array (and every cell map) lives in one padded
// layout, element (i,j,k) at i + px*j + sz*k with px >= nx+1 a multiple of
// 32 and sz = px*(ny+1); a thread "owns" the staggered entries whose lower
// corner is cell (i,j,k).  Entries on PEC walls are never written (they stay
// zero: tangential E, normal H, Sec. 3.2.3); periodic axes wrap the index.
//
// The bulk stencils march along z with the previous plane's values kept in
// registers, so each field value is fetched from HBM once per pass (x is
// the 64-lane wavefront direction; y and x neighbours come from L1/L2).
// Magnetic faces are handled from a compact face list: hm_pre builds the
// iteration-invariant quantities of eq:llg_tra5/6 and eq:iterate_H and does
// iteration r = 1 (which needs only H^s); h_bulk applies the non-magnetic
// Faraday update to every face; hm_iter is a cooperative persistent kernel
// that commits the magnetic H, then runs Jacobi iterations r = 2, 3, ...
// with a grid-wide max of |dM|/Ms after each one, all on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>
#include <stdint.h>

namespace mmk {

constexpr double kMu0 = 1.25663706212e-6;
constexpr double kEps0 = 8.8541878128e-12;

struct Geo {
  int nx, ny, nz;
  int px;        // x pitch (elements)
  int sz;        // z plane stride = px * (ny + 1)
  int per;       // bit 0/1/2: x/y/z periodic
  double dx, dy, dz;     // spacings
  double idx, idy, idz;  // 1/dx, 1/dy, 1/dz
};

// Difference quotient.  FP64 divides (the operation order of the reference
// definition, so FP64 results are reproducible to the bit); the FP32 bulk
// mode multiplies by the reciprocal spacing.
__device__ __forceinline__ double dq(double x, double d, double) { return x / d; }
__device__ __forceinline__ float dq(float x, float, float id) { return x * id; }

// Soft source restricted to the bounding box of its nonzero edges: J0 p is
// stored densely over the box (x fastest) and enters Step 2 as
// E = ca E + cb (curl H - J0 p g(t^{n+1/2})).
struct Src {
  const double* prof;     // dense over the box, or null
  int comp;
  int lo[3], hi[3];       // box [lo, hi) in staggered indices
  double g;               // g(t^{n+1/2})
};

__device__ __forceinline__ int at(const Geo& g, int i, int j, int k) {
  return i + g.px * j + g.sz * k;
}
// i-1 / i+1 along an axis of n cells; on a periodic axis the index wraps.
__device__ __forceinline__ int dn(int i, int n, bool per) { return (per && i == 0) ? n - 1 : i - 1; }
__device__ __forceinline__ int up(int i, int n, bool per) { return (per && i == n - 1) ? 0 : i + 1; }

template <typename T> __device__ __forceinline__ double D(T v) { return (double)v; }

// ---------------------------------------------------------------------------
// Step 2: E^{n+1} = ca E^n + cb curl H^{n+1/2} on interior edges, with eps and
// sigma on an edge the mean of its 4 cells and ca, cb from the time-centred
// Ampere law (Sec. 3.2.1, Step 2), with the soft current J^{n+1/2} fused in.
// Block 64 x 4 threads over (i, j); each thread marches k over [k0, k1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double src_term(const Src& s, int comp, int i, int j, int k) {
  if (!s.prof || comp != s.comp) return 0.0;
  if (i < s.lo[0] || i >= s.hi[0] || j < s.lo[1] || j >= s.hi[1] || k < s.lo[2] || k >= s.hi[2]) return 0.0;
  const int bx = s.hi[0] - s.lo[0], by = s.hi[1] - s.lo[1];
  return s.prof[(i - s.lo[0]) + bx * ((j - s.lo[1]) + by * (k - s.lo[2]))] * s.g;
}

template <typename T, bool SIG>
__global__ __launch_bounds__(256) void e_update(Geo g, T* __restrict__ Ex, T* __restrict__ Ey,
                                               T* __restrict__ Ez, const T* __restrict__ Hx,
                                               const T* __restrict__ Hy, const T* __restrict__ Hz,
                                               const T* __restrict__ eps, const T* __restrict__ sig,
                                               T dt, Src src, int kchunk) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(k0 + kchunk, g.nz);
  const bool iin = pxp || i >= 1;     // x node interior (Ey, Ez)
  const bool jin = pyp || j >= 1;     // y node interior (Ex, Ez)
  const int im = iin ? dn(i, g.nx, pxp) : i;   // clamped when unused: addresses stay valid
  const int jm = jin ? dn(j, g.ny, pyp) : j;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  const T e0 = (T)kEps0;
  const T half = (T)0.5, quarter = (T)0.25;

  // plane k-1 carries
  T hx_km = 0, hy_km = 0, e_km = 0, e_jm_km = 0, e_im_km = 0, s_km = 0, s_jm_km = 0, s_im_km = 0;
  if (pzp || k0 >= 1) {
    const int km = dn(k0, g.nz, pzp);
    hx_km = Hx[at(g, i, j, km)];
    hy_km = Hy[at(g, i, j, km)];
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
    const int cjm = at(g, i, jm, k);
    const int cim = at(g, im, j, k);
    const T hx = Hx[c], hy = Hy[c], hz = Hz[c];
    const T hz_jm = Hz[cjm], hx_jm = Hx[cjm];
    const T hz_im = Hz[cim], hy_im = Hy[cim];
    const T e_c = eps[c], e_jm = eps[cjm], e_im = eps[cim], e_imjm = eps[at(g, im, jm, k)];
    T s_c = 0, s_jm = 0, s_im = 0, s_imjm = 0;
    if (SIG) {
      s_c = sig[c];
      s_jm = sig[cjm];
      s_im = sig[cim];
      s_imjm = sig[at(g, im, jm, k)];
    }
    if (jin && kin) {  // Ex at (i+1/2, j, k)
      T curl = dq(hz - hz_jm, sdy, idy) - dq(hy - hy_km, sdz, idz);
      if (src.comp == 0) curl = curl - (T)src_term(src, 0, i, j, k);
      const T ee = e0 * (quarter * ((e_jm_km + e_km) + (e_jm + e_c)));
      const T a = ee / dt;
      const T b = SIG ? (quarter * ((s_jm_km + s_km) + (s_jm + s_c))) * half : (T)0;
      const T den = a + b;
      const T ca = SIG ? (a - b) / den : (T)1;
      const T cb = (T)1 / den;
      Ex[c] = ca * Ex[c] + cb * curl;
    }
    if (iin && kin) {  // Ey at (i, j+1/2, k)
      T curl = dq(hx - hx_km, sdz, idz) - dq(hz - hz_im, sdx, idx);
      if (src.comp == 1) curl = curl - (T)src_term(src, 1, i, j, k);
      const T ee = e0 * (quarter * ((e_im_km + e_km) + (e_im + e_c)));
      const T a = ee / dt;
      const T b = SIG ? (quarter * ((s_im_km + s_km) + (s_im + s_c))) * half : (T)0;
      const T den = a + b;
      const T ca = SIG ? (a - b) / den : (T)1;
      const T cb = (T)1 / den;
      Ey[c] = ca * Ey[c] + cb * curl;
    }
    if (iin && jin) {  // Ez at (i, j, k+1/2)
      T curl = dq(hy - hy_im, sdx, idx) - dq(hx - hx_jm, sdy, idy);
      if (src.comp == 2) curl = curl - (T)src_term(src, 2, i, j, k);
      const T ee = e0 * (quarter * ((e_imjm + e_jm) + (e_im + e_c)));
      const T a = ee / dt;
      const T b = SIG ? (quarter * ((s_imjm + s_jm) + (s_im + s_c))) * half : (T)0;
      const T den = a + b;
      const T ca = SIG ? (a - b) / den : (T)1;
      const T cb = (T)1 / den;
      Ez[c] = ca * Ez[c] + cb * curl;
    }
    hx_km = hx;
    hy_km = hy;
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

// ---------------------------------------------------------------------------
// H half step with the non-magnetic Faraday law (eq:Faraday3 with the local
// mu, Sec. 3.2.2): H <- H - (dt/2 mu_f) curl E on every interior face.
// Magnetic faces are overwritten afterwards by hm_iter.
// ---------------------------------------------------------------------------
template <typename T, bool MU>
__global__ __launch_bounds__(256) void h_bulk(Geo g, T* __restrict__ Hx, T* __restrict__ Hy,
                                             T* __restrict__ Hz, const T* __restrict__ Ex,
                                             const T* __restrict__ Ey, const T* __restrict__ Ez,
                                             const T* __restrict__ mu, T coef0, T h, int kchunk) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(k0 + kchunk, g.nz);
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
    const T ex_kp = Ex[at(g, i, j, kp)];
    const T ey_kp = Ey[at(g, i, j, kp)];
    const T ez = Ez[c];
    const T ez_jp = Ez[at(g, i, jp, k)];
    const T ez_ip = Ez[at(g, ip, j, k)];
    const T ey_ip = Ey[at(g, ip, j, k)];
    const T ex_jp = Ex[at(g, i, jp, k)];
    T mu_c = 0;
    if (MU) mu_c = mu[c];
    if (iin) {
      const T curl = dq(ez_jp - ez, sdy, idy) - dq(ey_kp - ey_k, sdz, idz);
      const T cf = MU ? h / (mu0 * (half * (mu[at(g, im, j, k)] + mu_c))) : coef0;
      Hx[c] = Hx[c] - cf * curl;
    }
    if (jin) {
      const T curl = dq(ex_kp - ex_k, sdz, idz) - dq(ez_ip - ez, sdx, idx);
      const T cf = MU ? h / (mu0 * (half * (mu[at(g, i, jm, k)] + mu_c))) : coef0;
      Hy[c] = Hy[c] - cf * curl;
    }
    if (pzp || k >= 1) {
      const T curl = dq(ey_ip - ey_k, sdx, idx) - dq(ex_jp - ex_k, sdy, idy);
      const T cf = MU ? h / (mu0 * (half * (mu_km + mu_c))) : coef0;
      Hz[c] = Hz[c] - cf * curl;
    }
    ex_k = ex_kp;
    ey_k = ey_kp;
    if (MU) mu_km = mu_c;
  }
}

// ---------------------------------------------------------------------------
// Magnetic faces (compact list; families 0, 1, 2 stored contiguously).
// ---------------------------------------------------------------------------
template <typename T>
struct Fields {
  T* E[3];
  T* H[3];
};

struct Mag {
  const int* idx;       // padded index of the face
  const double* Ms;     // face Ms
  const double* kap;    // mu0 * gamma_f * dt / 4 (signed gamma)
  const double* aoms;   // alpha_f / Ms_f
  double* M[3];         // current iterate (components x, y, z)
  double* b[3];         // b of eq:llg_tra6 (signed-gamma form), per sub-step
  double* d[3];         // (alpha/Ms) M^s, per sub-step
  double* q;            // H^s_n + M^s_n - (dt/2 mu0) curl E, per sub-step
  double* hnew;         // H^{(r)}_n of the latest iteration
  int off1, off2, n;    // family offsets and the number of evolving faces
};

__device__ __forceinline__ void face_ijk(const Geo& g, int c, int& i, int& j, int& k) {
  k = c / g.sz;
  const int r = c - k * g.sz;
  j = r / g.px;
  i = r - j * g.px;
}

// curl E at face (i,j,k) of family f.
template <typename T>
__device__ __forceinline__ double curl_e_face(const Geo& g, const Fields<T>& F, int f, int i, int j,
                                              int k) {
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const int c = at(g, i, j, k);
  if (f == 0) {
    const int jp = up(j, g.ny, pyp), kp = up(k, g.nz, pzp);
    return (D(F.E[2][at(g, i, jp, k)]) - D(F.E[2][c])) / g.dy -
           (D(F.E[1][at(g, i, j, kp)]) - D(F.E[1][c])) / g.dz;
  } else if (f == 1) {
    const int ip = up(i, g.nx, pxp), kp = up(k, g.nz, pzp);
    return (D(F.E[0][at(g, i, j, kp)]) - D(F.E[0][c])) / g.dz -
           (D(F.E[2][at(g, ip, j, k)]) - D(F.E[2][c])) / g.dx;
  } else {
    const int ip = up(i, g.nx, pxp), jp = up(j, g.ny, pyp);
    return (D(F.E[1][at(g, ip, j, k)]) - D(F.E[1][c])) / g.dx -
           (D(F.E[0][at(g, i, jp, k)]) - D(F.E[0][c])) / g.dy;
  }
}

// H_eff = H0 + H_EM at an interior face of family f: own normal H plus the
// two transverse components as four-point means (Sec. 3.1), each paired
// along the face normal first and then along the component's own axis.
template <typename T>
__device__ __forceinline__ void h_eff(const Geo& g, const Fields<T>& F, int f, int i, int j, int k,
                                      double H0x, double H0y, double H0z, double he[3]) {
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const int c = at(g, i, j, k);
  if (f == 0) {
    const int im = dn(i, g.nx, pxp), jp = up(j, g.ny, pyp), kp = up(k, g.nz, pzp);
    const T* Hy = F.H[1];
    const T* Hz = F.H[2];
    he[0] = D(F.H[0][c]) + H0x;
    he[1] = 0.25 * ((D(Hy[at(g, im, j, k)]) + D(Hy[c])) + (D(Hy[at(g, im, jp, k)]) + D(Hy[at(g, i, jp, k)]))) + H0y;
    he[2] = 0.25 * ((D(Hz[at(g, im, j, k)]) + D(Hz[c])) + (D(Hz[at(g, im, j, kp)]) + D(Hz[at(g, i, j, kp)]))) + H0z;
  } else if (f == 1) {
    const int jm = dn(j, g.ny, pyp), ip = up(i, g.nx, pxp), kp = up(k, g.nz, pzp);
    const T* Hx = F.H[0];
    const T* Hz = F.H[2];
    he[0] = 0.25 * ((D(Hx[at(g, i, jm, k)]) + D(Hx[c])) + (D(Hx[at(g, ip, jm, k)]) + D(Hx[at(g, ip, j, k)]))) + H0x;
    he[1] = D(F.H[1][c]) + H0y;
    he[2] = 0.25 * ((D(Hz[at(g, i, jm, k)]) + D(Hz[c])) + (D(Hz[at(g, i, jm, kp)]) + D(Hz[at(g, i, j, kp)]))) + H0z;
  } else {
    const int km = dn(k, g.nz, pzp), ip = up(i, g.nx, pxp), jp = up(j, g.ny, pyp);
    const T* Hx = F.H[0];
    const T* Hy = F.H[1];
    he[0] = 0.25 * ((D(Hx[at(g, i, j, km)]) + D(Hx[c])) + (D(Hx[at(g, ip, j, km)]) + D(Hx[at(g, ip, j, k)]))) + H0x;
    he[1] = 0.25 * ((D(Hy[at(g, i, j, km)]) + D(Hy[c])) + (D(Hy[at(g, i, jp, km)]) + D(Hy[at(g, i, jp, k)]))) + H0y;
    he[2] = D(F.H[2][c]) + H0z;
  }
}

// One closed-form trapezoidal LLG solve (eq:llg_tra4) followed by N(M):
// a = kappa H_eff - d, x = (b + (a.b) a - a x b) / (1 + |a|^2), M = x Ms/|x|.
__device__ __forceinline__ void llg_solve(const double he[3], double kap, const double d[3],
                                          const double b[3], double Ms, double m[3]) {
  double a[3];
  a[0] = kap * he[0] - d[0];
  a[1] = kap * he[1] - d[1];
  a[2] = kap * he[2] - d[2];
  const double ab = (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
  const double cx = a[1] * b[2] - a[2] * b[1];
  const double cy = a[2] * b[0] - a[0] * b[2];
  const double cz = a[0] * b[1] - a[1] * b[0];
  const double den = 1.0 + ((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]);
  const double x0 = (b[0] + ab * a[0] - cx) / den;
  const double x1 = (b[1] + ab * a[1] - cy) / den;
  const double x2 = (b[2] + ab * a[2] - cz) / den;
  const double nrm = sqrt((x0 * x0 + x1 * x1) + x2 * x2);
  const double s = Ms / nrm;
  m[0] = x0 * s;
  m[1] = x1 * s;
  m[2] = x2 * s;
}

// Residual bits: |dM|/Ms >= 0 is ordered like its IEEE bit pattern, and a NaN
// (sign cleared) compares above +Inf, so a uint64 max propagates it.
__device__ __forceinline__ unsigned long long rbits(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v) {
  __shared__ unsigned long long wmax[16];
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wmax[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int q = 1; q < nw; ++q) v = wmax[q] > v ? wmax[q] : v;
  }
  return v;   // valid in thread 0
}

__device__ __forceinline__ int face_family(const Mag& m, int t) {
  return t < m.off1 ? 0 : (t < m.off2 ? 1 : 2);
}

// Sub-step set-up and iteration r = 1 (which only needs H^s).
template <typename T>
__global__ __launch_bounds__(256) void hm_pre(Geo g, Fields<T> F, Mag m, double hmu0, double H0x,
                                             double H0y, double H0z,
                                             unsigned long long* __restrict__ res1) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long rb = 0;
  if (t < m.n) {
    const int f = face_family(m, t);
    const int c = m.idx[t];
    int i, j, k;
    face_ijk(g, c, i, j, k);
    const double C = curl_e_face(g, F, f, i, j, k);
    double he[3];
    h_eff(g, F, f, i, j, k, H0x, H0y, H0z, he);
    const double Ms = m.Ms[t], kap = m.kap[t], aoms = m.aoms[t];
    const double ms[3] = {m.M[0][t], m.M[1][t], m.M[2][t]};
    // M^s x H_eff^s
    const double mx = ms[1] * he[2] - ms[2] * he[1];
    const double my = ms[2] * he[0] - ms[0] * he[2];
    const double mz = ms[0] * he[1] - ms[1] * he[0];
    const double b[3] = {ms[0] + kap * mx, ms[1] + kap * my, ms[2] + kap * mz};
    const double d[3] = {aoms * ms[0], aoms * ms[1], aoms * ms[2]};
    const double q = D(F.H[f][c]) + ms[f] - hmu0 * C;
    double mn[3];
    llg_solve(he, kap, d, b, Ms, mn);
    const double hn = q - mn[f];
    double r = fabs(mn[0] - ms[0]) / Ms;
    unsigned long long bits = rbits(r);
    unsigned long long b1 = rbits(fabs(mn[1] - ms[1]) / Ms);
    unsigned long long b2 = rbits(fabs(mn[2] - ms[2]) / Ms);
    bits = b1 > bits ? b1 : bits;
    bits = b2 > bits ? b2 : bits;
    rb = bits;
    for (int q3 = 0; q3 < 3; ++q3) {
      m.b[q3][t] = b[q3];
      m.d[q3][t] = d[q3];
      m.M[q3][t] = mn[q3];
    }
    m.q[t] = q;
    m.hnew[t] = hn;
  }
  rb = block_max_u64(rb);
  if (threadIdx.x == 0 && rb) atomicMax(res1, rb);
}

__device__ __forceinline__ unsigned long long load_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Iterations r = 2, 3, ... of the H-M sub-step (Jacobi: every face reads its
// neighbours' H^{(r-1)}), with the grid-wide stopping test of Sec. 3.2.2
// after each one.  Cooperative launch; every wave reaches each grid.sync and
// the loop ends after at most max(max_iter, fixed_iter) iterations.
template <typename T>
__global__ __launch_bounds__(256) void hm_iter(Geo g, Fields<T> F, Mag m, double H0x, double H0y,
                                              double H0z, unsigned long long* __restrict__ res,
                                              unsigned long long* __restrict__ res_next, int nres,
                                              double tol, int max_iter, int fixed_iter,
                                              int* __restrict__ iters_out, int* __restrict__ err) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  if (blockIdx.x == 0)
    for (int s = threadIdx.x; s < nres; s += blockDim.x) res_next[s] = 0ull;
  for (int t = tid; t < m.n; t += nth) F.H[face_family(m, t)][m.idx[t]] = (T)m.hnew[t];
  __threadfence();
  grid.sync();
  __threadfence();
  int r = 1;
  double rv = 0.0;
  for (;;) {
    rv = __longlong_as_double((long long)load_u64(&res[r]));
    const bool bad = !(rv <= 1.0e308);          // NaN or +Inf
    bool stop;
    if (bad) stop = true;
    else if (fixed_iter > 0) stop = r >= fixed_iter;
    else stop = (rv < tol) || (r >= max_iter);
    if (stop) break;
    ++r;
    unsigned long long lb = 0;
    for (int t = tid; t < m.n; t += nth) {
      const int f = face_family(m, t);
      const int c = m.idx[t];
      int i, j, k;
      face_ijk(g, c, i, j, k);
      double he[3];
      h_eff(g, F, f, i, j, k, H0x, H0y, H0z, he);
      const double Ms = m.Ms[t];
      const double d[3] = {m.d[0][t], m.d[1][t], m.d[2][t]};
      const double b[3] = {m.b[0][t], m.b[1][t], m.b[2][t]};
      const double mo[3] = {m.M[0][t], m.M[1][t], m.M[2][t]};
      double mn[3];
      llg_solve(he, m.kap[t], d, b, Ms, mn);
      m.hnew[t] = m.q[t] - mn[f];
      for (int q3 = 0; q3 < 3; ++q3) {
        m.M[q3][t] = mn[q3];
        const unsigned long long bb = rbits(fabs(mn[q3] - mo[q3]) / Ms);
        lb = bb > lb ? bb : lb;
      }
    }
    lb = block_max_u64(lb);
    if (threadIdx.x == 0 && lb) atomicMax(&res[r], lb);
    __threadfence();
    grid.sync();
    __threadfence();
    for (int t = tid; t < m.n; t += nth) F.H[face_family(m, t)][m.idx[t]] = (T)m.hnew[t];
    __threadfence();
    grid.sync();
    __threadfence();
  }
  if (tid == 0) {
    iters_out[0] = r;
    const bool bad = !(rv <= 1.0e308);
    if (bad) atomicOr(err, 2);
    else if (fixed_iter <= 0 && !(rv < tol)) atomicOr(err, 1);
  }
}

// ---------------------------------------------------------------------------
// Probes (FP64 accumulation).
// ---------------------------------------------------------------------------
struct PointProbe {
  int slot;             // series row
  const void* h;        // field array (T) or null
  const double* mcomp;  // compact M component or null
  int ih, im;           // indices
  double ch, cm;        // value = ch * h[ih] + cm * mcomp[im]
};

template <typename T>
__global__ void probe_points(const PointProbe* __restrict__ pp, int np, double* __restrict__ series,
                            size_t cap, double* __restrict__ sums, long step, double dt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const PointProbe q = pp[p];
  double v = 0.0;
  if (q.h) v += q.ch * D(((const T*)q.h)[q.ih]);
  if (q.mcomp) v += q.cm * q.mcomp[q.im];
  series[(size_t)q.slot * cap + step] = v;
  sums[q.slot] += dt * v;
}

// Poynting flux through the node plane x = i0: deterministic two-level sum
// (fixed per-thread strides, fixed tree, partials combined in block order by
// the last block to finish).
template <typename T>
__global__ __launch_bounds__(256) void probe_flux(Geo g, Fields<T> F, const int* __restrict__ planes,
                                                 const int* __restrict__ slots, double* __restrict__ partial,
                                                 unsigned int* __restrict__ ticket,
                                                 double* __restrict__ series, size_t cap,
                                                 double* __restrict__ sums, long step, double dt,
                                                 double dydz, int NY, int NZ) {
  const int p = blockIdx.y;
  const int i0 = planes[p];
  const bool pxp = g.per & 1;
  const int im = dn(i0, g.nx, pxp);
  const int nb = gridDim.x;
  // Ey*Hz over j in [0,ny), k in [0,NZ); Ez*Hy over j in [0,NY), k in [0,nz)
  const int n1 = g.ny * NZ, n2 = NY * g.nz;
  double s1 = 0.0, s2 = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n1; e += nb * blockDim.x) {
    const int k = e / g.ny, j = e - k * g.ny;
    const double hz = 0.5 * (D(F.H[2][at(g, im, j, k)]) + D(F.H[2][at(g, i0, j, k)]));
    s1 += D(F.E[1][at(g, i0, j, k)]) * hz;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += nb * blockDim.x) {
    const int k = e / NY, j = e - k * NY;
    const double hy = 0.5 * (D(F.H[1][at(g, im, j, k)]) + D(F.H[1][at(g, i0, j, k)]));
    s2 += D(F.E[2][at(g, i0, j, k)]) * hy;
  }
  __shared__ double r1[256], r2[256];
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  __shared__ bool last;
  if (threadIdx.x == 0) {
    partial[(size_t)p * 2 * nb + 2 * blockIdx.x] = r1[0];
    partial[(size_t)p * 2 * nb + 2 * blockIdx.x + 1] = r2[0];
    __threadfence();
    const unsigned int tk = atomicAdd(&ticket[p], 1u);
    last = (tk == (unsigned)nb - 1);
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    double a = 0.0, b = 0.0;
    const double* pp = partial + (size_t)p * 2 * nb;
    for (int q = 0; q < nb; ++q) {
      a += __hip_atomic_load(&pp[2 * q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      b += __hip_atomic_load(&pp[2 * q + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const double P = dydz * (a - b);
    series[(size_t)slots[p] * cap + step] = P;
    sums[slots[p]] += dt * P;
    ticket[p] = 0u;
  }
}

}  // namespace mmk
