// Device kernels of the coupled Maxwell-LLG step for gfx950 (CDNA4).
//
// Scheme: Yao, Jambunathan, Zeng & Nonaka, Sec. 3.2.2 (second-order coupled
// scheme) on the Yee grid of Sec. 3.1.  One step is
//   Step 1: H-M sub-step with curl E^n     (hm_pre -> h_bulk -> hm_step.. -> hm_finish -> hm_commit)
//   Step 2: E update with the soft source   (e_update)
//   Step 3: H-M sub-step with curl E^{n+1} (the same sequence)
//   probes at level n+1                     (probe_points, probe_flux, probe_flux_sum)
// This file holds that per-iteration form of the H-M sub-step; grids with
// many magnetic faces take the fused form of hm_fused.h (h_half_db ->
// hm_fused -> hm_more, the same results).  Inside one mm_step call the
// tiles away from magnetic faces take Step 3 of one step and Step 1 of the
// next in one pass (h_bulk with NP = 2), which also fills the flux planes'
// capture the probe reads.
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
// Faraday update to every face; the Jacobi iterations r = 2, 3, ... then
// ping-pong the magnetic faces' H between H and a shadow array A (odd r
// write A, even r write H; non-magnetic neighbours are always read from H),
// so an iteration needs no commit pass.  They run as ordinary launches
// (hm_step) that return at once when the device-side stopping test on the
// max of |dM|/Ms has fired; hm_finish continues the iteration if the
// launches enqueued were too few, and hm_commit brings the final H home.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

// Threads per block of the magnetic-face kernels (hm_pre, hm_step,
// hm_commit) and the cap on their blocks per CU: the grid of those launches
// is also the number of residual partials each consumer reduces.
#ifndef MM_MAG_THREADS
#define MM_MAG_THREADS 256
#endif
#ifndef MM_MAG_BLOCKS_PER_CU
#define MM_MAG_BLOCKS_PER_CU 4
#endif

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

// A bulk launch runs over tiles of 64 x 4 columns x kc planes taken from a
// list, so the host chooses which tiles run and which XCD (block id mod 8)
// each lands on.  Tile id = bx + gx (by + gy bz).  With split > 1 each tile
// is cut along z into `split` runs of ceil(kc / split) planes, one block
// each (blocks b = split * q + s: tile list[q], run s), for launches over
// too few tiles to fill the chip.  An e_update launch with blockDim.y = 8
// takes two tiles stacked in y per block (the list holds the lower one), so
// one block streams both tiles' rows at each plane; the upper tile's y halo
// is the lower tile's last row.  Measured 2 % faster than single tiles on
// the 512 x 256 x 256 grid, for slightly more HBM reads.
struct Tiles {
  const int* list;
  int gx, gy, kc, split;
};

// Origin (i0, j0) and plane range [k0, k1) of this block's run (empty
// when the tile is shorter than the run's start).
__device__ __forceinline__ void tile_span(const Tiles& t, int nz, int& i0, int& j0, int& k0, int& k1) {
  const int q = blockIdx.x / t.split, s = blockIdx.x - q * t.split;
  const int id = t.list[q];
  const int bx = id % t.gx, r = id / t.gx;
  const int ks = (t.kc + t.split - 1) / t.split;
  const int kt = (r / t.gy) * t.kc;
  i0 = bx * 64;
  j0 = (r % t.gy) * 4;
  k0 = kt + s * ks;
  k1 = min(min(k0 + ks, kt + t.kc), nz);
}

// ---------------------------------------------------------------------------
// Step 2: E^{n+1} = ca E^n + cb curl H^{n+1/2} on interior edges, with eps and
// sigma on an edge the mean of its 4 cells and ca, cb from the time-centred
// Ampere law (Sec. 3.2.1, Step 2), with the soft current J^{n+1/2} fused in.
// Block 64 x 4 threads over (i, j) of one tile; each thread marches k over
// the tile's planes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double src_term(const Src& s, int comp, int i, int j, int k) {
  if (!s.prof || comp != s.comp) return 0.0;
  if (i < s.lo[0] || i >= s.hi[0] || j < s.lo[1] || j >= s.hi[1] || k < s.lo[2] || k >= s.hi[2]) return 0.0;
  const int bx = s.hi[0] - s.lo[0], by = s.hi[1] - s.lo[1];
  return s.prof[(i - s.lo[0]) + bx * ((j - s.lo[1]) + by * (k - s.lo[2]))] * s.g;
}

// MAT: the cell maps come as a byte material id per cell and a table of
// (eps_r, sigma) per id (exactly the values of the dense maps), staged in
// LDS: 1 byte per cell instead of two map values.
// OOP: E^{n+1} goes to (Ox, Oy, Oz) and E^n stays in (Ex, Ey, Ez) (the
// adjoint's recompute keeps every level); only interior edges are written.
template <typename T, bool SIG, bool MAT, int RY = 4, bool OOP = false>
__global__ __launch_bounds__(64 * RY) void e_update(Geo g, T* __restrict__ Ex, T* __restrict__ Ey,
                                               T* __restrict__ Ez, const T* __restrict__ Hx,
                                               const T* __restrict__ Hy, const T* __restrict__ Hz,
                                               const T* __restrict__ eps_map, const T* __restrict__ sig_map,
                                               const unsigned char* __restrict__ mat,
                                               const T* __restrict__ mtab, T dt, Src src, Tiles tl,
                                               T* __restrict__ Ox, T* __restrict__ Oy, T* __restrict__ Oz) {
  // Edge coefficients of an edge whose four cells share one material,
  // per material id: the same expressions as the general path below (so
  // equal to it bit for bit); mixed edges take the general path.
  auto coef = [&](T e1, T e2, T e3, T e4, T s1, T s2, T s3, T s4, T& ca, T& cb) {
    const T ee = (T)kEps0 * ((T)0.25 * ((e1 + e2) + (e3 + e4)));
    const T a = ee / dt;
    const T b = SIG ? ((T)0.25 * ((s1 + s2) + (s3 + s4))) * (T)0.5 : (T)0;
    const T den = a + b;
    ca = SIG ? (a - b) / den : (T)1;
    cb = (T)1 / den;
  };
  __shared__ T teps[MAT ? 256 : 1], tsig[MAT ? 256 : 1], tca[MAT ? 256 : 1], tcb[MAT ? 256 : 1];
  if (MAT) {
    const int q = threadIdx.x + 64 * threadIdx.y;
    if (q < 256) {
      const T e = mtab[q], sg = mtab[256 + q];
      teps[q] = e;
      tsig[q] = sg;
      coef(e, e, e, e, sg, sg, sg, sg, tca[q], tcb[q]);
    }
    __syncthreads();
  }
  int i, j, k0, k1;
  tile_span(tl, g.nz, i, j, k0, k1);
  i += threadIdx.x;
  j += threadIdx.y;
  if (i >= g.nx || j >= g.ny || k0 >= k1) return;
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const bool iin = pxp || i >= 1;     // x node interior (Ey, Ez)
  const bool jin = pyp || j >= 1;     // y node interior (Ex, Ez)
  const int im = iin ? dn(i, g.nx, pxp) : i;   // clamped when unused: addresses stay valid
  const int jm = jin ? dn(j, g.ny, pyp) : j;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  // plane k-1 carries
  T hx_km = 0, hy_km = 0, e_km = 0, e_jm_km = 0, e_im_km = 0, s_km = 0, s_jm_km = 0, s_im_km = 0;
  int m_km = -1, m_jm_km = -1, m_im_km = -1;   // material ids of plane k-1 (MAT)
  if (pzp || k0 >= 1) {
    const int km = dn(k0, g.nz, pzp);
    if (MAT) {
      m_km = mat[at(g, i, j, km)];
      m_jm_km = mat[at(g, i, jm, km)];
      m_im_km = mat[at(g, im, j, km)];
    }
    hx_km = Hx[at(g, i, j, km)];
    hy_km = Hy[at(g, i, j, km)];
    if (!MAT) {
      e_km = eps_map[at(g, i, j, km)];
      e_jm_km = eps_map[at(g, i, jm, km)];
      e_im_km = eps_map[at(g, im, j, km)];
      if (SIG) {
        s_km = sig_map[at(g, i, j, km)];
        s_jm_km = sig_map[at(g, i, jm, km)];
        s_im_km = sig_map[at(g, im, j, km)];
      }
    }
  }
  // Software pipeline over the planes: every load of plane k+1 (H and its
  // neighbours, the old E, the materials) is issued before plane k is
  // computed, so one memory latency per plane overlaps the work.  (The
  // source profile is read where it is used: only blocks inside its
  // bounding box do.)
  struct Plane {
    T hx, hy, hz, hz_jm, hx_jm, hz_im, hy_im, ex, ey, ez;
    T e_c, e_jm, e_im, e_imjm, s_c, s_jm, s_im, s_imjm;
    int m_c, m_jm, m_im, m_imjm;
  };
  auto load = [&](int k, Plane& p) {
    const int c = at(g, i, j, k), cjm = at(g, i, jm, k), cim = at(g, im, j, k), cimjm = at(g, im, jm, k);
    p.hx = Hx[c];
    p.hy = Hy[c];
    p.hz = Hz[c];
    p.hz_jm = Hz[cjm];
    p.hx_jm = Hx[cjm];
    p.hz_im = Hz[cim];
    p.hy_im = Hy[cim];
    p.ex = Ex[c];
    p.ey = Ey[c];
    p.ez = Ez[c];
    if (MAT) {
      p.m_c = mat[c];
      p.m_jm = mat[cjm];
      p.m_im = mat[cim];
      p.m_imjm = mat[cimjm];
    } else {
      p.e_c = eps_map[c];
      p.e_jm = eps_map[cjm];
      p.e_im = eps_map[cim];
      p.e_imjm = eps_map[cimjm];
      if (SIG) {
        p.s_c = sig_map[c];
        p.s_jm = sig_map[cjm];
        p.s_im = sig_map[cim];
        p.s_imjm = sig_map[cimjm];
      }
    }
  };
  Plane nxt;
  load(k0, nxt);
  for (int k = k0; k < k1; ++k) {
    const Plane cur = nxt;
    if (k + 1 < k1) load(k + 1, nxt);
    __builtin_amdgcn_sched_barrier(0);
    const bool kin = pzp || k >= 1;
    const int c = at(g, i, j, k);
    // cell eps_r / sigma: from the LDS table by id (MAT; read only where an
    // edge is mixed) or the values loaded from the maps
    auto EV = [&](int id, T v) -> T { return MAT ? teps[id] : v; };
    auto SV = [&](int id, T v) -> T { return SIG ? (MAT ? tsig[id] : v) : (T)0; };
    // (the four cells of each edge, in the pairing order of the 4-cell mean)
    if (jin && kin) {  // Ex at (i+1/2, j, k)
      T curl = dq(cur.hz - cur.hz_jm, sdy, idy) - dq(cur.hy - hy_km, sdz, idz);
      if (src.comp == 0) curl = curl - (T)src_term(src, 0, i, j, k);
      T ca, cb;
      if (MAT && m_jm_km == m_km && m_km == cur.m_jm && cur.m_jm == cur.m_c) {
        ca = tca[cur.m_c];
        cb = tcb[cur.m_c];
      } else {
        coef(EV(m_jm_km, e_jm_km), EV(m_km, e_km), EV(cur.m_jm, cur.e_jm), EV(cur.m_c, cur.e_c),
             SV(m_jm_km, s_jm_km), SV(m_km, s_km), SV(cur.m_jm, cur.s_jm), SV(cur.m_c, cur.s_c), ca, cb);
      }
      (OOP ? Ox : Ex)[c] = ca * cur.ex + cb * curl;
    }
    if (iin && kin) {  // Ey at (i, j+1/2, k)
      T curl = dq(cur.hx - hx_km, sdz, idz) - dq(cur.hz - cur.hz_im, sdx, idx);
      if (src.comp == 1) curl = curl - (T)src_term(src, 1, i, j, k);
      T ca, cb;
      if (MAT && m_im_km == m_km && m_km == cur.m_im && cur.m_im == cur.m_c) {
        ca = tca[cur.m_c];
        cb = tcb[cur.m_c];
      } else {
        coef(EV(m_im_km, e_im_km), EV(m_km, e_km), EV(cur.m_im, cur.e_im), EV(cur.m_c, cur.e_c),
             SV(m_im_km, s_im_km), SV(m_km, s_km), SV(cur.m_im, cur.s_im), SV(cur.m_c, cur.s_c), ca, cb);
      }
      (OOP ? Oy : Ey)[c] = ca * cur.ey + cb * curl;
    }
    if (iin && jin) {  // Ez at (i, j, k+1/2)
      T curl = dq(cur.hy - cur.hy_im, sdx, idx) - dq(cur.hx - cur.hx_jm, sdy, idy);
      if (src.comp == 2) curl = curl - (T)src_term(src, 2, i, j, k);
      T ca, cb;
      if (MAT && cur.m_imjm == cur.m_jm && cur.m_jm == cur.m_im && cur.m_im == cur.m_c) {
        ca = tca[cur.m_c];
        cb = tcb[cur.m_c];
      } else {
        coef(EV(cur.m_imjm, cur.e_imjm), EV(cur.m_jm, cur.e_jm), EV(cur.m_im, cur.e_im), EV(cur.m_c, cur.e_c),
             SV(cur.m_imjm, cur.s_imjm), SV(cur.m_jm, cur.s_jm), SV(cur.m_im, cur.s_im), SV(cur.m_c, cur.s_c),
             ca, cb);
      }
      (OOP ? Oz : Ez)[c] = ca * cur.ez + cb * curl;
    }
    hx_km = cur.hx;
    hy_km = cur.hy;
    if (MAT) {
      m_km = cur.m_c;
      m_jm_km = cur.m_jm;
      m_im_km = cur.m_im;
    } else {
      e_km = cur.e_c;
      e_jm_km = cur.e_jm;
      e_im_km = cur.e_im;
      if (SIG) {
        s_km = cur.s_c;
        s_jm_km = cur.s_jm;
        s_im_km = cur.s_im;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// H half step with the non-magnetic Faraday law (eq:Faraday3 with the local
// mu, Sec. 3.2.2): H <- H - (dt/2 mu_f) curl E on every interior face.
// Magnetic faces are overwritten afterwards by the iteration.
//
// NP = 2 applies two half steps with the same curl E in registers: Step 3
// of step n and Step 1 of step n+1 both use curl E^{n+1}, so on tiles that
// hold no magnetic face and no face an H_eff of a magnetic face reads, the
// two passes fuse into one.  Each half step is the same rounded
// subtraction, so the result equals two NP = 1 launches bit for bit.
//
// With NP = 2 the pass also passes through H^{n+1}, the level the probes
// sample.  For up to kCapPlanes flux planes x = i0 it stores what the
// Poynting flux (Sec. 5.2) needs from these tiles densely per plane node
// (j, k): E_y, E_z at i0 and H_y, H_z at i0 - 1 and i0 at level n+1, so the
// probe reads a few contiguous arrays instead of one cache line per value
// of x-fastest fields.
// ---------------------------------------------------------------------------
constexpr int kCapPlanes = 4;
constexpr int kCapPlanesZ = 32;   // tile depth the capture allows
template <typename T>
struct FluxCap {
  T* buf;                  // [plane][6][NY][NZ]: Ey(i0), Ez(i0), Hy(im), Hz(im), Hy(i0), Hz(i0); null: off
  int n;                   // planes captured (distinct x)
  int i0[kCapPlanes];      // plane x node
  int im[kCapPlanes];      // the x face before it (wrapped on a periodic x axis)
  int NZ;                  // plane nodes along z
  long long nn;            // plane nodes, NY * NZ
};

// Capture roles of one wave (one x row of 64 columns from tx, at one j): the
// lane whose column is x = i0 of a plane and the lane whose column is its
// x = im (or -1), with the offsets of node (j, k0) in that plane's capture;
// all wave-uniform.  During a z-march the capture lanes park their values in
// LDS (no global store inside a pipelined loop); afterwards the wave writes
// them out, one lane per plane (runs of at most kCapPlanesZ planes).
struct CapRole {
  int l0, lm;
  long long o0, om;
};

template <typename T>
__device__ __forceinline__ CapRole cap_role(const FluxCap<T>& cap, int tx, int j, int k0) {
  CapRole r{-1, -1, 0, 0};
  if (!cap.buf) return r;
  const long long jw = __builtin_amdgcn_readfirstlane(j);
  for (int p = 0; p < cap.n; ++p) {
    const long long b = (long long)p * 6 * cap.nn + jw * cap.NZ + k0;
    if (cap.i0[p] >= tx && cap.i0[p] < tx + 64) {
      r.l0 = cap.i0[p] - tx;
      r.o0 = b;
    }
    if (cap.im[p] >= tx && cap.im[p] < tx + 64) {
      r.lm = cap.im[p] - tx;
      r.om = b + 2 * cap.nn;
    }
  }
  return r;
}

// Park plane kk's values (E_y, E_z at i0; H_y, H_z at level n+1) in the
// wave's stash st (6 x kCapPlanesZ).
template <typename T>
__device__ __forceinline__ void cap_park(const CapRole& r, T* st, int kk, T ey, T ez, T hy, T hz) {
  if ((int)threadIdx.x == r.l0) {
    st[kk] = ey;
    st[kCapPlanesZ + kk] = ez;
    st[4 * kCapPlanesZ + kk] = hy;
    st[5 * kCapPlanesZ + kk] = hz;
  }
  if ((int)threadIdx.x == r.lm) {
    st[2 * kCapPlanesZ + kk] = hy;
    st[3 * kCapPlanesZ + kk] = hz;
  }
}

// Write the n parked planes out (every lane of the wave takes part).
template <typename T>
__device__ __forceinline__ void cap_flush(const CapRole& r, const FluxCap<T>& cap, const T* st, int n) {
  // the LDS writes came from other lanes of this wave
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int kk = threadIdx.x;   // node (j, k0 + kk): consecutive lanes, consecutive addresses
  if (kk < n) {
    if (r.l0 >= 0) {
      cap.buf[r.o0 + kk] = st[kk];
      cap.buf[r.o0 + cap.nn + kk] = st[kCapPlanesZ + kk];
      cap.buf[r.o0 + 4 * cap.nn + kk] = st[4 * kCapPlanesZ + kk];
      cap.buf[r.o0 + 5 * cap.nn + kk] = st[5 * kCapPlanesZ + kk];
    }
    if (r.lm >= 0) {
      cap.buf[r.om + kk] = st[2 * kCapPlanesZ + kk];
      cap.buf[r.om + cap.nn + kk] = st[3 * kCapPlanesZ + kk];
    }
  }
}

template <typename T, bool MU, int NP>
__global__ __launch_bounds__(256) void h_bulk(Geo g, T* __restrict__ Hx, T* __restrict__ Hy,
                                             T* __restrict__ Hz, const T* __restrict__ Ex,
                                             const T* __restrict__ Ey, const T* __restrict__ Ez,
                                             const T* __restrict__ mu, T coef0, T h, Tiles tl,
                                             FluxCap<T> cap = {}) {
  int i, j, k0, k1;
  tile_span(tl, g.nz, i, j, k0, k1);
  const int tx = i;
  i += threadIdx.x;
  j += threadIdx.y;
  // flux-plane capture (see CapRole)
  __shared__ T stash[NP == 2 ? 4 * 6 * kCapPlanesZ : 1];
  CapRole cr{-1, -1, 0, 0};
  if (NP == 2) cr = cap_role(cap, tx, j, k0);
  if (j >= g.ny || k0 >= k1) return;
  const bool capw = NP == 2 && (cr.l0 >= 0 || cr.lm >= 0);   // wave-uniform
  T* st = stash + (NP == 2 ? __builtin_amdgcn_readfirstlane(threadIdx.y) * 6 * kCapPlanesZ : 0);
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

  // Software pipeline over the planes (as in e_update): plane k+1's loads
  // are issued before plane k is computed.
  struct Plane {
    T ex_kp, ey_kp, ez, ez_jp, ez_ip, ey_ip, ex_jp, hx, hy, hz, mu_c, mu_im, mu_jm;
  };
  auto load = [&](int k, Plane& p) {
    const int kp = up(k, g.nz, pzp);
    const int c = at(g, i, j, k);
    p.ex_kp = Ex[at(g, i, j, kp)];
    p.ey_kp = Ey[at(g, i, j, kp)];
    p.ez = Ez[c];
    p.ez_jp = Ez[at(g, i, jp, k)];
    p.ez_ip = Ez[at(g, ip, j, k)];
    p.ey_ip = Ey[at(g, ip, j, k)];
    p.ex_jp = Ex[at(g, i, jp, k)];
    p.hx = Hx[c];
    p.hy = Hy[c];
    p.hz = Hz[c];
    if (MU) {
      p.mu_c = mu[c];
      p.mu_im = mu[at(g, im, j, k)];
      p.mu_jm = mu[at(g, i, jm, k)];
    }
  };
  T ex_k = Ex[at(g, i, j, k0)];
  T ey_k = Ey[at(g, i, j, k0)];
  T mu_km = 0;
  if (MU && (pzp || k0 >= 1)) mu_km = mu[at(g, i, j, dn(k0, g.nz, pzp))];
  Plane nxt;
  load(k0, nxt);
  for (int k = k0; k < k1; ++k) {
    const Plane cur = nxt;
    if (k + 1 < k1) load(k + 1, nxt);
    __builtin_amdgcn_sched_barrier(0);
    const int c = at(g, i, j, k);
    T hy1 = cur.hy, hz1 = cur.hz;   // level n+1, after the first half step
    if (iin) {
      const T curl = dq(cur.ez_jp - cur.ez, sdy, idy) - dq(cur.ey_kp - ey_k, sdz, idz);
      const T cf = MU ? h / (mu0 * (half * (cur.mu_im + cur.mu_c))) : coef0;
      T v = cur.hx;
      for (int p = 0; p < NP; ++p) v = v - cf * curl;
      Hx[c] = v;
    }
    if (jin) {
      const T curl = dq(cur.ex_kp - ex_k, sdz, idz) - dq(cur.ez_ip - cur.ez, sdx, idx);
      const T cf = MU ? h / (mu0 * (half * (cur.mu_jm + cur.mu_c))) : coef0;
      T v = cur.hy - cf * curl;
      hy1 = v;
      for (int p = 1; p < NP; ++p) v = v - cf * curl;
      Hy[c] = v;
    }
    if (pzp || k >= 1) {
      const T curl = dq(cur.ey_ip - ey_k, sdx, idx) - dq(cur.ex_jp - ex_k, sdy, idy);
      const T cf = MU ? h / (mu0 * (half * (mu_km + cur.mu_c))) : coef0;
      T v = cur.hz - cf * curl;
      hz1 = v;
      for (int p = 1; p < NP; ++p) v = v - cf * curl;
      Hz[c] = v;
    }
    if (capw) cap_park(cr, st, k - k0, ey_k, cur.ez, hy1, hz1);   // E and H at level n+1
    ex_k = cur.ex_kp;
    ey_k = cur.ey_kp;
    if (MU) mu_km = cur.mu_c;
  }
  }
  if (capw) cap_flush(cr, cap, st, k1 - k0);
}

// ---------------------------------------------------------------------------
// Open boundary (Sec. 3.2.3): split-field perfectly matched layer on the
// tiles that hold layer entries.  Component c splits into the part driven by
// the positive term of its curl, P (derivative along axis p), and the rest
// (axis m): x: p = y, m = z;  y: p = z, m = x;  z: p = x, m = y.  The full
// field stays in E / H and P in a side array.  In the layer (damping rate
// kappa > 0 along p or m at the entry) each part takes the macroscopic
// update and is multiplied by the damping factor of its axis before and
// after it: exp(-kappa dt/2) for E, exp(-kappa dt/4) for each H half step.
// Other entries take the plain update of e_update / h_bulk (the same
// arithmetic, so the same bits).
// ---------------------------------------------------------------------------
template <typename T>
struct Pml {
  const double* dn[3];          // E factor at the nodes of axis a
  const double* dc[3];          // H factor at the cell centres of axis a
  const unsigned char* on_n[3];  // kappa > 0 at the nodes of axis a
  const unsigned char* on_c[3];  // kappa > 0 at the cell centres of axis a
  T* PE[3];
  T* PH[3];
};

template <typename T, bool SIG>
__global__ __launch_bounds__(256) void pml_e(Geo g, T* __restrict__ Ex, T* __restrict__ Ey, T* __restrict__ Ez,
                                            const T* __restrict__ Hx, const T* __restrict__ Hy,
                                            const T* __restrict__ Hz, const T* __restrict__ eps,
                                            const T* __restrict__ sig, T dt, Src src, Tiles tl, Pml<T> P) {
  int i, j, k0, k1;
  tile_span(tl, g.nz, i, j, k0, k1);
  i += threadIdx.x;
  j += threadIdx.y;
  if (i >= g.nx || j >= g.ny || k0 >= k1) return;
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const bool iin = pxp || i >= 1, jin = pyp || j >= 1;
  const int im = iin ? dn(i, g.nx, pxp) : i;
  const int jm = jin ? dn(j, g.ny, pyp) : j;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  auto coef = [&](T e1, T e2, T e3, T e4, T s1, T s2, T s3, T s4, T& ca, T& cb) {
    const T ee = (T)kEps0 * ((T)0.25 * ((e1 + e2) + (e3 + e4)));
    const T a = ee / dt;
    const T b = SIG ? ((T)0.25 * ((s1 + s2) + (s3 + s4))) * (T)0.5 : (T)0;
    const T den = a + b;
    ca = SIG ? (a - b) / den : (T)1;
    cb = (T)1 / den;
  };
  auto S = [&](int a) -> T { return SIG ? sig[a] : (T)0; };
  // one component: plain update, or the split update in the layer
  auto upd = [&](T* E, T* PE, int c, T tp, T tm, T sv, T ca, T cb, double dpv, double dmv, bool on) {
    if (!on) {
      T curl = tp - tm;
      curl = curl - sv;
      E[c] = ca * E[c] + cb * curl;
    } else {
      const T dp = (T)dpv, dm = (T)dmv;
      const T pv = PE[c], mv = E[c] - pv;
      const T pn = dp * (ca * (dp * pv) + cb * (tp - sv));
      const T mn = dm * (ca * (dm * mv) - cb * tm);
      PE[c] = pn;
      E[c] = pn + mn;
    }
  };
  for (int k = k0; k < k1; ++k) {
    const bool kin = pzp || k >= 1;
    const int km = kin ? dn(k, g.nz, pzp) : k;
    const int c = at(g, i, j, k), cjm = at(g, i, jm, k), cim = at(g, im, j, k), ckm = at(g, i, j, km);
    if (jin && kin) {  // Ex: p = y (node j), m = z (node k)
      const T tp = dq(Hz[c] - Hz[cjm], sdy, idy), tm = dq(Hy[c] - Hy[ckm], sdz, idz);
      const T sv = src.comp == 0 ? (T)src_term(src, 0, i, j, k) : (T)0;
      T ca, cb;
      coef(eps[at(g, i, jm, km)], eps[ckm], eps[cjm], eps[c], S(at(g, i, jm, km)), S(ckm), S(cjm), S(c), ca, cb);
      upd(Ex, P.PE[0], c, tp, tm, sv, ca, cb, P.dn[1][j], P.dn[2][k], P.on_n[1][j] || P.on_n[2][k]);
    }
    if (iin && kin) {  // Ey: p = z (node k), m = x (node i)
      const T tp = dq(Hx[c] - Hx[ckm], sdz, idz), tm = dq(Hz[c] - Hz[cim], sdx, idx);
      const T sv = src.comp == 1 ? (T)src_term(src, 1, i, j, k) : (T)0;
      T ca, cb;
      coef(eps[at(g, im, j, km)], eps[ckm], eps[cim], eps[c], S(at(g, im, j, km)), S(ckm), S(cim), S(c), ca, cb);
      upd(Ey, P.PE[1], c, tp, tm, sv, ca, cb, P.dn[2][k], P.dn[0][i], P.on_n[2][k] || P.on_n[0][i]);
    }
    if (iin && jin) {  // Ez: p = x (node i), m = y (node j)
      const T tp = dq(Hy[c] - Hy[cim], sdx, idx), tm = dq(Hx[c] - Hx[cjm], sdy, idy);
      const T sv = src.comp == 2 ? (T)src_term(src, 2, i, j, k) : (T)0;
      T ca, cb;
      coef(eps[at(g, im, jm, k)], eps[cjm], eps[cim], eps[c], S(at(g, im, jm, k)), S(cjm), S(cim), S(c), ca, cb);
      upd(Ez, P.PE[2], c, tp, tm, sv, ca, cb, P.dn[0][i], P.dn[1][j], P.on_n[0][i] || P.on_n[1][j]);
    }
  }
}

// One H half step on the layer tiles (every face, like h_bulk with NP = 1;
// magnetic faces there are overwritten by the iteration afterwards).
template <typename T, bool MU>
__global__ __launch_bounds__(256) void pml_h(Geo g, T* __restrict__ Hx, T* __restrict__ Hy, T* __restrict__ Hz,
                                            const T* __restrict__ Ex, const T* __restrict__ Ey,
                                            const T* __restrict__ Ez, const T* __restrict__ mu, T coef0, T h,
                                            Tiles tl, Pml<T> P) {
  int i, j, k0, k1;
  tile_span(tl, g.nz, i, j, k0, k1);
  i += threadIdx.x;
  j += threadIdx.y;
  if (i >= g.nx || j >= g.ny || k0 >= k1) return;
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const bool iin = pxp || i >= 1, jin = pyp || j >= 1;
  const int ip = up(i, g.nx, pxp), jp = up(j, g.ny, pyp);
  const int im = iin ? dn(i, g.nx, pxp) : i;
  const int jm = jin ? dn(j, g.ny, pyp) : j;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  const T mu0 = (T)kMu0, half = (T)0.5;
  auto upd = [&](T* H, T* PH, int c, T tp, T tm, T cf, double dpv, double dmv, bool on) {
    if (!on) {
      const T curl = tp - tm;
      H[c] = H[c] - cf * curl;
    } else {
      const T dp = (T)dpv, dm = (T)dmv;
      const T pv = PH[c], mv = H[c] - pv;
      const T pn = dp * (dp * pv - cf * tp);
      const T mn = dm * (dm * mv + cf * tm);
      PH[c] = pn;
      H[c] = pn + mn;
    }
  };
  for (int k = k0; k < k1; ++k) {
    const int kp = up(k, g.nz, pzp);
    const int c = at(g, i, j, k);
    if (iin) {  // Hx: p = y (centre j), m = z (centre k)
      const T tp = dq(Ez[at(g, i, jp, k)] - Ez[c], sdy, idy), tm = dq(Ey[at(g, i, j, kp)] - Ey[c], sdz, idz);
      const T cf = MU ? h / (mu0 * (half * (mu[at(g, im, j, k)] + mu[c]))) : coef0;
      upd(Hx, P.PH[0], c, tp, tm, cf, P.dc[1][j], P.dc[2][k], P.on_c[1][j] || P.on_c[2][k]);
    }
    if (jin) {  // Hy: p = z (centre k), m = x (centre i)
      const T tp = dq(Ex[at(g, i, j, kp)] - Ex[c], sdz, idz), tm = dq(Ez[at(g, ip, j, k)] - Ez[c], sdx, idx);
      const T cf = MU ? h / (mu0 * (half * (mu[at(g, i, jm, k)] + mu[c]))) : coef0;
      upd(Hy, P.PH[1], c, tp, tm, cf, P.dc[2][k], P.dc[0][i], P.on_c[2][k] || P.on_c[0][i]);
    }
    if (pzp || k >= 1) {  // Hz: p = x (centre i), m = y (centre j)
      const int km = dn(k, g.nz, pzp);
      const T tp = dq(Ey[at(g, ip, j, k)] - Ey[c], sdx, idx), tm = dq(Ex[at(g, i, jp, k)] - Ex[c], sdy, idy);
      const T cf = MU ? h / (mu0 * (half * (mu[at(g, i, j, km)] + mu[c]))) : coef0;
      upd(Hz, P.PH[2], c, tp, tm, cf, P.dc[0][i], P.dc[1][j], P.on_c[0][i] || P.on_c[1][j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Magnetic faces (compact list; families 0, 1, 2 stored contiguously).
// ---------------------------------------------------------------------------
template <typename T>
struct Fields {
  T* E[3];
  T* H[3];
  T* A[3];   // shadow H on magnetic faces: iterates r = 1, 4, 7, ...
  T* B[3];   // second shadow: iterates r = 2, 5, 8, ...; r = 3, 6, ... go to H
};

// Three component pointers held in registers.  A per-thread component index
// picks one with selects: indexing a pointer array in memory by a value that
// varies across the wavefront would turn every access into a dependent
// load of the pointer first.
template <typename T>
struct Tri {
  T* p0;
  T* p1;
  T* p2;
  __device__ __forceinline__ T* operator()(int f) const { return f == 0 ? p0 : (f == 1 ? p1 : p2); }
};

template <typename T>
__device__ __forceinline__ Tri<T> tri(T* const (&a)[3]) {
  return Tri<T>{a[0], a[1], a[2]};
}

// Where iteration r writes H on the evolving faces.  The iterates rotate
// through A, B and H: iteration r reads r-1 from the previous buffer while
// no thread reads the one it writes (the faces of H it writes are read by
// nobody in that iteration: other faces' reads of evolving neighbours go to
// the previous iterate), and the usual count of 3 ends in H itself.
template <typename T>
__device__ __forceinline__ Tri<T> iter_buf(const Fields<T>& F, int r) {
  const int q = r % 3;
  return q == 1 ? tri(F.A) : (q == 2 ? tri(F.B) : tri(F.H));
}

struct Mag {
  const int* idx;            // padded index of the face
  const unsigned char* nbm;  // bit q: transverse neighbour q is an evolving magnetic face
  const double* Ms;          // face Ms
  const double* kap;         // mu0 * gamma_f * dt / 4 (signed gamma)
  const double* aoms;        // alpha_f / Ms_f
  const unsigned char* fid;  // or null: per face an id into ftab, which holds
  const double* ftab;        // (Ms, kap, aoms) per id (the same values, 1 byte per face)
  double* M[3];              // current iterate (components x, y, z)
  double* b[3];              // b of eq:llg_tra6 (signed-gamma form), per sub-step
  double* d[3];              // (alpha/Ms) M^s, per sub-step
  double* q;                 // H^s_n + M^s_n - (dt/2 mu0) curl E, per sub-step
  double* hlog;              // optional: H^{(r)} of every face, slot r-1 (for the adjoint)
  int hlog_cap;              // number of slots in hlog
  int off1, off2, n;         // family offsets and the number of evolving faces
};

// Record H^{(r)} of face t in the iterate log (adjoint recompute only).
__device__ __forceinline__ void log_iterate(const Mag& m, int r, int t, double v, int* err) {
  if (!m.hlog) return;
  if (r <= m.hlog_cap) m.hlog[(size_t)(r - 1) * m.n + t] = v;
  else atomicOr(err, 8);
}

// The face constants of evolving face t: from the per-face arrays, or by the
// face's material id from the table.
__device__ __forceinline__ void face_consts(const Mag& m, int t, double& Ms, double& kap, double& aoms) {
  if (m.fid) {
    const double* e = m.ftab + 3 * (int)m.fid[t];
    Ms = e[0];
    kap = e[1];
    aoms = e[2];
  } else {
    Ms = m.Ms[t];
    kap = m.kap[t];
    aoms = m.aoms[t];
  }
}

__device__ __forceinline__ void face_ijk(const Geo& g, int c, int& i, int& j, int& k) {
  k = c / g.sz;
  const int r = c - k * g.sz;
  j = r / g.px;
  i = r - j * g.px;
}

// curl E at face (i,j,k) of family f (FP64, reference operation order).
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

// Where iteration r reads H^{(r-1)}: evolving magnetic faces from `alt`
// (bit q of `mask` set for transverse neighbour q), all other faces from
// `base`.  With alt == base every read comes from one array.
template <typename T>
struct HRead {
  const T* base[3];
  const T* alt[3];
  unsigned mask;
  __device__ __forceinline__ double v(int comp, int c, int q) const {
    return D(((mask >> q) & 1u) ? alt[comp][c] : base[comp][c]);
  }
};

// H_eff = H0 + H_EM at an interior face of family f: own normal H plus the
// two transverse components as four-point means (Sec. 3.1), each paired
// along the face normal first and then along the component's own axis.
// Neighbour q numbering: first transverse component q = 0..3, second 4..7,
// in the order (f-1, c), (f, c), (f-1, c+1), (f, c+1).
//
// Split into the eight gathers (h_eff_load) and the sums (h_eff_sum) so a
// kernel can issue every load of a face before the first use.
template <typename T>
__device__ __forceinline__ void h_eff_load(const Geo& g, const HRead<T>& R, int f, int i, int j, int k,
                                           double v[8]) {
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const int c = at(g, i, j, k);
  if (f == 0) {
    const int im = dn(i, g.nx, pxp), jp = up(j, g.ny, pyp), kp = up(k, g.nz, pzp);
    v[0] = R.v(1, at(g, im, j, k), 0);
    v[1] = R.v(1, c, 1);
    v[2] = R.v(1, at(g, im, jp, k), 2);
    v[3] = R.v(1, at(g, i, jp, k), 3);
    v[4] = R.v(2, at(g, im, j, k), 4);
    v[5] = R.v(2, c, 5);
    v[6] = R.v(2, at(g, im, j, kp), 6);
    v[7] = R.v(2, at(g, i, j, kp), 7);
  } else if (f == 1) {
    const int jm = dn(j, g.ny, pyp), ip = up(i, g.nx, pxp), kp = up(k, g.nz, pzp);
    v[0] = R.v(0, at(g, i, jm, k), 0);
    v[1] = R.v(0, c, 1);
    v[2] = R.v(0, at(g, ip, jm, k), 2);
    v[3] = R.v(0, at(g, ip, j, k), 3);
    v[4] = R.v(2, at(g, i, jm, k), 4);
    v[5] = R.v(2, c, 5);
    v[6] = R.v(2, at(g, i, jm, kp), 6);
    v[7] = R.v(2, at(g, i, j, kp), 7);
  } else {
    const int km = dn(k, g.nz, pzp), ip = up(i, g.nx, pxp), jp = up(j, g.ny, pyp);
    v[0] = R.v(0, at(g, i, j, km), 0);
    v[1] = R.v(0, c, 1);
    v[2] = R.v(0, at(g, ip, j, km), 2);
    v[3] = R.v(0, at(g, ip, j, k), 3);
    v[4] = R.v(1, at(g, i, j, km), 4);
    v[5] = R.v(1, c, 5);
    v[6] = R.v(1, at(g, i, jp, km), 6);
    v[7] = R.v(1, at(g, i, jp, k), 7);
  }
}

__device__ __forceinline__ void h_eff_sum(const double v[8], double own, int f, double H0x, double H0y,
                                          double H0z, double he[3]) {
  const double t1 = 0.25 * ((v[0] + v[1]) + (v[2] + v[3]));
  const double t2 = 0.25 * ((v[4] + v[5]) + (v[6] + v[7]));
  if (f == 0) {
    he[0] = own + H0x;
    he[1] = t1 + H0y;
    he[2] = t2 + H0z;
  } else if (f == 1) {
    he[0] = t1 + H0x;
    he[1] = own + H0y;
    he[2] = t2 + H0z;
  } else {
    he[0] = t1 + H0x;
    he[1] = t2 + H0y;
    he[2] = own + H0z;
  }
}

template <typename T>
__device__ __forceinline__ void h_eff(const Geo& g, const HRead<T>& R, double own, int f, int i, int j,
                                      int k, double H0x, double H0y, double H0z, double he[3]) {
  double v[8];
  h_eff_load(g, R, f, i, j, k, v);
  h_eff_sum(v, own, f, H0x, H0y, H0z, he);
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

// Max over the block, returned in every thread.
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v) {
  __shared__ unsigned long long wmax[16];
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wmax[w] = v;
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  v = wmax[0];
  for (int q = 1; q < nw; ++q) v = wmax[q] > v ? wmax[q] : v;
  __syncthreads();
  return v;
}

__device__ __forceinline__ int face_family(const Mag& m, int t) {
  return t < m.off1 ? 0 : (t < m.off2 ? 1 : 2);
}

__device__ __forceinline__ unsigned long long load_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-sub-step control (one per sub-step parity).  The residual of
// iteration r is the max of P per-block partials part[r * P + b], each
// written with a plain store by block b of the launch that ran iteration r
// (every slot is written every time, so nothing needs clearing); whoever
// needs the residual reduces the P partials itself.  One device-scope atomic
// per block on a single address would serialise across the XCDs (~11 ns
// each, 140 us for a 12k-block launch).
//   cur[0]   the final iteration count once the stopping rule has fired (0 before)
struct Ctl {
  unsigned long long* cur;
  unsigned long long* next;   // the other sub-step's cur, cleared by hm_commit
  unsigned long long* part;   // partial maxima of this sub-step, P per iteration
  int P;
  double tol;
  int max_iter, fixed_iter;
};

// Block-wide: the residual bits of iteration r (all threads get the value).
__device__ __forceinline__ unsigned long long residual_bits(const Ctl& C, int r) {
  const unsigned long long* p = C.part + (size_t)r * C.P;
  unsigned long long v = 0;
  for (int q = threadIdx.x; q < C.P; q += blockDim.x) {
    const unsigned long long w = load_u64(&p[q]);
    v = w > v ? w : v;
  }
  return block_max_u64(v);
}

// Block-wide: publish this block's residual bits of iteration r.  A grid
// smaller than P also fills the slots no block of it owns.
__device__ __forceinline__ void publish_residual(const Ctl& C, int r, unsigned long long lb) {
  lb = block_max_u64(lb);
  unsigned long long* p = C.part + (size_t)r * C.P;
  if (threadIdx.x == 0)
    for (int q = blockIdx.x; q < C.P; q += gridDim.x)
      __hip_atomic_store(&p[q], q == (int)blockIdx.x ? lb : 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stopping rule of Sec. 3.2.2 after iteration r_done, given its residual
// bits: stop on a non-finite residual, on residual < tol, at max_iter, or
// (fixed mode) after fixed_iter iterations.
__device__ __forceinline__ bool stop_rule(const Ctl& C, int r_done, unsigned long long bits, bool& bad) {
  const double rv = __longlong_as_double((long long)bits);
  bad = !(rv <= 1.0e308);
  if (bad) return true;
  if (C.fixed_iter > 0) return r_done >= C.fixed_iter;
  return (rv < C.tol) || (r_done >= C.max_iter);
}

// One Jacobi iteration r >= 2 for the faces t = t0, t0 + stride, ...; reads
// H^{(r-1)} through `Rd` and writes H^{(r)} into `out`.  Returns the max of
// the residual bits.
template <typename T>
__device__ __forceinline__ unsigned long long iterate_faces(const Geo& g, const Mag& m, const Fields<T>& F,
                                                            Tri<T> prev, Tri<T> out, int t0, int stride,
                                                            double H0x, double H0y, double H0z, int r,
                                                            int* err) {
  unsigned long long lb = 0;
  for (int t = t0; t < m.n; t += stride) {
    // batch 1: everything indexed by the face number
    const int f = face_family(m, t);
    const int c = m.idx[t];
    const unsigned mask = m.nbm[t];
    double Ms, kap, aoms_unused;
    face_consts(m, t, Ms, kap, aoms_unused);
    const double qf = m.q[t];
    const double d[3] = {m.d[0][t], m.d[1][t], m.d[2][t]};
    const double b[3] = {m.b[0][t], m.b[1][t], m.b[2][t]};
    const double mo[3] = {m.M[0][t], m.M[1][t], m.M[2][t]};
    __builtin_amdgcn_sched_barrier(0);
    // batch 2: the face's own H^{(r-1)} and its eight neighbours
    int i, j, k;
    face_ijk(g, c, i, j, k);
    HRead<T> Rd;
    Rd.base[0] = F.H[0];
    Rd.base[1] = F.H[1];
    Rd.base[2] = F.H[2];
    Rd.alt[0] = prev.p0;
    Rd.alt[1] = prev.p1;
    Rd.alt[2] = prev.p2;
    Rd.mask = mask;
    double nv[8];
    const double own = D(prev(f)[c]);
    h_eff_load(g, Rd, f, i, j, k, nv);
    __builtin_amdgcn_sched_barrier(0);
    double he[3];
    h_eff_sum(nv, own, f, H0x, H0y, H0z, he);
    double mn[3];
    llg_solve(he, kap, d, b, Ms, mn);
    const T hv = (T)(qf - mn[f]);
    out(f)[c] = hv;
    log_iterate(m, r, t, D(hv), err);
    for (int q3 = 0; q3 < 3; ++q3) {
      m.M[q3][t] = mn[q3];
      const unsigned long long bb = rbits(fabs(mn[q3] - mo[q3]) / Ms);
      lb = bb > lb ? bb : lb;
    }
  }
  return lb;
}

// Sub-step set-up and iteration r = 1 (which only needs H^s): the
// iteration-invariant b, d of eq:llg_tra5/6 and q of eq:iterate_H, then
// M^{(1)} in place and H^{(1)} into the shadow array A.
//
// first != 0: the first-order scheme of Sec. 3.2.1 instead.  M^{new} =
// N(M^s + h [k1 M^s x H_eff^s + k2 M^s x (M^s x H_eff^s)]) with the face
// constants k1 = mu0 gamma_L, k2 = alpha mu0 gamma_L / Ms held in kap and
// aoms (eq:LLG_scalar, gamma_L = gamma / (1 + alpha^2)), then H from
// eq:H_update as in iteration 1; the sub-step ends there.
template <typename T>
__global__ __launch_bounds__(MM_MAG_THREADS) void hm_pre(Geo g, Fields<T> F, Mag m, double h, double hmu0, double H0x,
                                             double H0y, double H0z, int first, Ctl C, int* err) {
  unsigned long long rb = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m.n; t += gridDim.x * blockDim.x) {
    // batch 1: everything indexed by the face number
    const int f = face_family(m, t);
    const int c = m.idx[t];
    double Ms, kap, aoms;
    face_consts(m, t, Ms, kap, aoms);
    const double ms[3] = {m.M[0][t], m.M[1][t], m.M[2][t]};
    __builtin_amdgcn_sched_barrier(0);
    // batch 2: curl E and H^s around the face
    int i, j, k;
    face_ijk(g, c, i, j, k);
    const double Cf = curl_e_face(g, F, f, i, j, k);
    HRead<T> Rd;
    Rd.base[0] = Rd.alt[0] = F.H[0];
    Rd.base[1] = Rd.alt[1] = F.H[1];
    Rd.base[2] = Rd.alt[2] = F.H[2];
    Rd.mask = 0;
    const double hs = D(tri(F.H)(f)[c]);
    double nv[8];
    h_eff_load(g, Rd, f, i, j, k, nv);
    __builtin_amdgcn_sched_barrier(0);
    double he[3];
    h_eff_sum(nv, hs, f, H0x, H0y, H0z, he);
    // M^s x H_eff^s
    const double mx = ms[1] * he[2] - ms[2] * he[1];
    const double my = ms[2] * he[0] - ms[0] * he[2];
    const double mz = ms[0] * he[1] - ms[1] * he[0];
    const double q = hs + ms[f] - hmu0 * Cf;
    double mn[3];
    if (first) {
      const double k1 = kap, k2 = aoms;
      const double xx = ms[1] * mz - ms[2] * my;
      const double xy = ms[2] * mx - ms[0] * mz;
      const double xz = ms[0] * my - ms[1] * mx;
      const double mt[3] = {ms[0] + h * (k1 * mx + k2 * xx), ms[1] + h * (k1 * my + k2 * xy),
                            ms[2] + h * (k1 * mz + k2 * xz)};
      const double nrm = sqrt((mt[0] * mt[0] + mt[1] * mt[1]) + mt[2] * mt[2]);
      const double s = Ms / nrm;
      mn[0] = mt[0] * s;
      mn[1] = mt[1] * s;
      mn[2] = mt[2] * s;
    } else {
      const double b[3] = {ms[0] + kap * mx, ms[1] + kap * my, ms[2] + kap * mz};
      const double d[3] = {aoms * ms[0], aoms * ms[1], aoms * ms[2]};
      llg_solve(he, kap, d, b, Ms, mn);
      for (int q3 = 0; q3 < 3; ++q3) {
        m.b[q3][t] = b[q3];
        m.d[q3][t] = d[q3];
      }
    }
    const T hv = (T)(q - mn[f]);
    tri(F.A)(f)[c] = hv;
    log_iterate(m, 1, t, D(hv), err);
    for (int q3 = 0; q3 < 3; ++q3) {
      const unsigned long long bb = rbits(fabs(mn[q3] - ms[q3]) / Ms);
      rb = bb > rb ? bb : rb;
      m.M[q3][t] = mn[q3];
    }
    m.q[t] = q;
  }
  publish_residual(C, 1, rb);
}

// Iteration r >= 2 as an ordinary launch.  Every thread evaluates the
// stopping rule on iteration r-1's residual (the same value everywhere) and
// the whole grid returns at once when it fires; block 0 then records the
// final count.  H^{(r)} goes where iter_buf puts it.
template <typename T>
__global__ __launch_bounds__(MM_MAG_THREADS) void hm_step(Geo g, Fields<T> F, Mag m, double H0x, double H0y,
                                              double H0z, Ctl C, int r, int* err) {
  if (load_u64(&C.cur[0]) != 0ull) return;
  bool bad;
  if (stop_rule(C, r - 1, residual_bits(C, r - 1), bad)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) C.cur[0] = (unsigned long long)(r - 1);
    return;
  }
  const Tri<T> prev = iter_buf(F, r - 1);
  const Tri<T> out = iter_buf(F, r);
  const unsigned long long lb = iterate_faces(g, m, F, prev, out, blockIdx.x * blockDim.x + threadIdx.x,
                                              gridDim.x * blockDim.x, H0x, H0y, H0z, r, err);
  publish_residual(C, r, lb);
}

// Bounded-spin barrier across the (small, co-resident) grid of hm_finish.
// bar[0] arrival count, bar[1] generation.  Returns false on timeout.
__device__ __forceinline__ bool grid_barrier(unsigned int* bar) {
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    __threadfence();
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (atomicAdd(&bar[0], 1u) == gridDim.x - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      atomicAdd(&bar[1], 1u);
    } else {
      long n = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++n > 10000000L) {
          ok = 0;
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
  return ok != 0;
}

// If the launches enqueued have not met the stopping rule, keep iterating
// here (one barrier per iteration; the grid is at most one block per CU, so
// it is resident as a whole).  Either way ctl[0] ends holding the final
// count.  Returns at once in the common case.
template <typename T>
__global__ __launch_bounds__(256) void hm_finish(Geo g, Fields<T> F, Mag m, double H0x, double H0y,
                                                double H0z, Ctl C, int r_next, unsigned int* bar, int* err) {
  if (load_u64(&C.cur[0]) != 0ull) return;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  bool bad = false;
  int r = r_next;
  for (;;) {
    if (stop_rule(C, r - 1, residual_bits(C, r - 1), bad)) break;
    const Tri<T> prev = iter_buf(F, r - 1);
    const Tri<T> out = iter_buf(F, r);
    const unsigned long long lb = iterate_faces(g, m, F, prev, out, tid, nth, H0x, H0y, H0z, r, err);
    publish_residual(C, r, lb);
    if (!grid_barrier(bar)) {
      if (threadIdx.x == 0) atomicOr(err, 4);
      r += 1;
      break;
    }
    ++r;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) C.cur[0] = (unsigned long long)(r - 1);
}

// End of a sub-step: bring the final magnetic H into H when it sits in A or
// B (a count that is not a multiple of 3), record the count and the sticky
// flags, and clear the other sub-step's final count.
template <typename T>
__global__ __launch_bounds__(MM_MAG_THREADS) void hm_commit(Fields<T> F, Mag m, Ctl C, int* iters_out, int* ring,
                                                int* err) {
  const int rfin = (int)load_u64(&C.cur[0]);
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (rfin % 3 != 0) {
    const Tri<T> src = iter_buf(F, rfin);
    for (int t = tid; t < m.n; t += gridDim.x * blockDim.x) {
      const int f = face_family(m, t);
      const int c = m.idx[t];
      tri(F.H)(f)[c] = src(f)[c];
    }
  }
  if (blockIdx.x == 0) {
    const unsigned long long bits = residual_bits(C, rfin);
    if (threadIdx.x == 0) {
      C.next[0] = 0ull;
      iters_out[0] = rfin;
      ring[0] = rfin;
      bool bad;
      stop_rule(C, rfin, bits, bad);
      int e = 0;
      if (bad) e |= 2;
      else if (C.fixed_iter <= 0) {
        const double rv = __longlong_as_double((long long)bits);
        if (!(rv < C.tol)) e |= 1;
      }
      if (e) atomicOr(err, e);
    }
  }
}

// ---------------------------------------------------------------------------
// Probes (FP64 accumulation).
// ---------------------------------------------------------------------------

// Within a multi-step run the tiles that take the fused two-half-step H
// update hold H^{n+1/2} when the probes of level n+1 are taken.  Lag tells
// the probes which tiles those are (far[tile] != 0; far == null: none) and
// how h_bulk would have advanced them.
template <typename T>
struct Lag {
  const unsigned char* far;
  const T* Hn[3];  // or null: where the other (near) tiles' H is, during a fused run
  const T* mu;    // cell mu_r, or null when mu_r = 1 everywhere
  T coef0, h;     // dt / (2 mu0) and dt / 2
  int gx, gy, kc;
};

// H at face (f, i, j, k) at the probe level: the stored value, or for a
// lagging tile the Faraday half step with the current E applied to it with
// exactly the arithmetic of h_bulk (so the probe sees the value a separate
// half-step pass would have stored).
template <typename T>
__device__ double h_level(const Geo& g, const Fields<T>& F, const Lag<T>& L, int f, int i, int j, int k) {
  const int c = at(g, i, j, k);
  const T hv = tri(F.H)(f)[c];
  if (i >= g.nx || j >= g.ny || k >= g.nz) return D(hv);   // PEC wall faces: zero in both buffers
  if (!L.far || !L.far[(i >> 6) + L.gx * ((j >> 2) + L.gy * (k / L.kc))])
    return L.Hn[0] ? D(L.Hn[f][c]) : D(hv);
  const bool pxp = g.per & 1, pyp = g.per & 2, pzp = g.per & 4;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const T sdx = (T)g.dx, sdy = (T)g.dy, sdz = (T)g.dz;
  const T mu0 = (T)kMu0, half = (T)0.5;
  const T* Ex = F.E[0];
  const T* Ey = F.E[1];
  const T* Ez = F.E[2];
  T curl, cf = L.coef0;
  if (f == 0) {
    if (!(pxp || i >= 1)) return D(hv);
    const int jp = up(j, g.ny, pyp), kp = up(k, g.nz, pzp);
    curl = dq(Ez[at(g, i, jp, k)] - Ez[c], sdy, idy) - dq(Ey[at(g, i, j, kp)] - Ey[c], sdz, idz);
    if (L.mu) cf = L.h / (mu0 * (half * (L.mu[at(g, dn(i, g.nx, pxp), j, k)] + L.mu[c])));
  } else if (f == 1) {
    if (!(pyp || j >= 1)) return D(hv);
    const int ip = up(i, g.nx, pxp), kp = up(k, g.nz, pzp);
    curl = dq(Ex[at(g, i, j, kp)] - Ex[c], sdz, idz) - dq(Ez[at(g, ip, j, k)] - Ez[c], sdx, idx);
    if (L.mu) cf = L.h / (mu0 * (half * (L.mu[at(g, i, dn(j, g.ny, pyp), k)] + L.mu[c])));
  } else {
    if (!(pzp || k >= 1)) return D(hv);
    const int ip = up(i, g.nx, pxp), jp = up(j, g.ny, pyp);
    curl = dq(Ey[at(g, ip, j, k)] - Ey[c], sdx, idx) - dq(Ex[at(g, i, jp, k)] - Ex[c], sdy, idy);
    if (L.mu) cf = L.h / (mu0 * (half * (L.mu[at(g, i, j, dn(k, g.nz, pzp))] + L.mu[c])));
  }
  return D((T)(hv - cf * curl));
}

struct PointProbe {
  int slot;             // series row
  const void* h;        // field array (T) or null
  const double* mcomp;  // compact M component or null
  int ih, im;           // indices
  double ch, cm;        // value = ch * h[ih] + cm * mcomp[im]
  int fam;              // h is H of this face family (read at the probe level), or -1
  int pi, pj, pk;       // (i, j, k) of entry ih
};

template <typename T>
__global__ void probe_points(Geo g, Fields<T> F, Lag<T> L, const PointProbe* __restrict__ pp, int np,
                            double* __restrict__ series, size_t cap, double* __restrict__ sums, long step,
                            double dt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const PointProbe q = pp[p];
  double v = 0.0;
  if (q.h) {
    const double hv = q.fam >= 0 ? h_level(g, F, L, q.fam, q.pi, q.pj, q.pk) : D(((const T*)q.h)[q.ih]);
    v += q.ch * hv;
  }
  if (q.mcomp) v += q.cm * q.mcomp[q.im];
  series[(size_t)q.slot * cap + step] = v;
  sums[q.slot] += dt * v;
}

// Poynting flux through the node plane x = i0: deterministic two-level sum.
// One thread per node (j, k) of the plane, z fastest, takes both terms there
// (E_y H_z for j < ny, k < NZ and E_z H_y for j < NY, k < nz), so the lines
// of the x-fastest arrays it touches serve both; a fixed tree per block into
// one partial per block, and probe_flux_sum adds the partials in a fixed
// order (a launch of its own: a last-block ticket needed a device-scope
// fence per block, which cost more than the launch).
//
// With a capture (FluxCap.buf set; the far tiles' fused pass has run and
// holds H^{n+3/2}), values at faces and edges of far tiles come from the
// capture that pass stored on its way through level n+1; the near tiles'
// values are read from the fields as without one, or, with near != 0 (the
// fused sub-step's last half step filled the capture as well), from the
// capture where it holds them.  fmask says which entries of a node the
// capture holds (bits 0-1 far tiles, 2-6 near tiles; fixed by the tile
// split and the magnetic faces).
template <typename T>
__global__ __launch_bounds__(256) void probe_flux(Geo g, Fields<T> F, Lag<T> L, const int* __restrict__ planes,
                                                 double* __restrict__ partial, int NY, int NZ, FluxCap<T> fc,
                                                 const unsigned char* __restrict__ fmask, int near) {
  const int p = blockIdx.y;
  const int i0 = planes[p];
  const bool pxp = g.per & 1;
  const int im = dn(i0, g.nx, pxp);
  const int nb = gridDim.x;
  double s1 = 0.0, s2 = 0.0;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < NY * NZ) {
    const int j = e / NZ, k = e - j * NZ;
    const T* cb = fc.buf ? fc.buf + (long long)p * 6 * fc.nn + e : nullptr;
    unsigned m = cb ? fmask[(long long)p * NY * NZ + e] : 0u;
    // per entry: far tile (bit 0 / 1) or, when the near tiles filled it, near
    m = (m & 3u) | (near ? (m & 124u) : 0u);
    const bool e0 = m & 5u;                              // E_y, E_z at i0
    const bool hy0c = m & 9u, hz0c = m & 17u;            // H at i0
    const bool hymc = m & 34u, hzmc = m & 66u;           // H at im
    if (j < g.ny) {
      const double hzm = hzmc ? D(cb[3 * fc.nn]) : h_level(g, F, L, 2, im, j, k);
      const double hz0 = hz0c ? D(cb[5 * fc.nn]) : h_level(g, F, L, 2, i0, j, k);
      const double hz = 0.5 * (hzm + hz0);
      s1 = (e0 ? D(cb[0]) : D(F.E[1][at(g, i0, j, k)])) * hz;
    }
    if (k < g.nz) {
      const double hym = hymc ? D(cb[2 * fc.nn]) : h_level(g, F, L, 1, im, j, k);
      const double hy0 = hy0c ? D(cb[4 * fc.nn]) : h_level(g, F, L, 1, i0, j, k);
      const double hy = 0.5 * (hym + hy0);
      s2 = (e0 ? D(cb[fc.nn]) : D(F.E[2][at(g, i0, j, k)])) * hy;
    }
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
  if (threadIdx.x == 0) {
    partial[(size_t)p * 2 * nb + 2 * blockIdx.x] = r1[0];
    partial[(size_t)p * 2 * nb + 2 * blockIdx.x + 1] = r2[0];
  }
}

// The plane sums of probe_flux (block p: plane p): thread t adds the
// partials t, t + 256, ... in order, then a fixed tree; P = dy dz (sum1 -
// sum2) into the series and dt P into the time integral.
__global__ __launch_bounds__(256) void probe_flux_sum(const double* __restrict__ partial, int nb,
                                                      const int* __restrict__ slots, double* __restrict__ series,
                                                      size_t cap, double* __restrict__ sums, long step, double dt,
                                                      double dydz) {
  const int p = blockIdx.x;
  const double* pp = partial + (size_t)p * 2 * nb;
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x) {
    a += pp[2 * q];
    b += pp[2 * q + 1];
  }
  __shared__ double r1[256], r2[256];
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double P = dydz * (r1[0] - r2[0]);
    series[(size_t)slots[p] * cap + step] = P;
    sums[slots[p]] += dt * P;
  }
}

// Hard source (Sec. 3.2): after an update of one E or H component, its
// entries in the box [lo, lo + n) of staggered indices take prof * g (the
// profile dense over the box, x fastest).  Entries pinned by a PEC wall
// (tangential E, normal H) keep their zero.  One thread per box entry.
struct Hard {
  const double* prof;
  int lo[3], n[3];
  int comp;               // 0-2: E component, 3-5: H family + 3
  double g;               // g at the level the update ends at
};

template <typename T>
__global__ __launch_bounds__(256) void hard_set(Geo g, T* f, Hard s) {
  const long long nb = (long long)s.n[0] * s.n[1] * s.n[2];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  const int bi = (int)(t % s.n[0]);
  const long long r = t / s.n[0];
  const int p[3] = {s.lo[0] + bi, s.lo[1] + (int)(r % s.n[1]), s.lo[2] + (int)(r / s.n[1])};
  const int n3[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    if ((g.per >> a) & 1) continue;
    // E_c is pinned on the walls normal to its other two axes, H_f on the
    // walls normal to f
    const bool wall_axis = s.comp < 3 ? a != s.comp : a == s.comp - 3;
    if (wall_axis && (p[a] == 0 || p[a] == n3[a])) return;
  }
  f[at(g, p[0], p[1], p[2])] = (T)(s.prof[t] * s.g);
}

}  // namespace mmk
