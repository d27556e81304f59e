// Host runtime and C ABI of the coupled Maxwell-LLG stepper (see include/mm.h).
//
// mm_init turns the cell-centred inputs into the device layout (padded
// field arrays, cell maps, the compact magnetic-face list with its
// per-face constants, the soft-source edge list); mm_step enqueues the
// kernel sequence of kernels.h on the context's stream; everything else is
// argument checking, staging copies and probe/statistics bookkeeping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/mm.h"
#include "kernels.h"
#include "hm_fused.h"
#include "adjoint.h"

using mmk::Geo;

// Fixed device storage of mm_step_noalloc (see resolve_scratch).
constexpr size_t kScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr double kC0 = 299792458.0;

struct ProbeRec {
  mm_probe_desc d;
  mmk::PointProbe pp;  // for kind 0
};

// The cells behind a magnetic face (for the Ms chain of the adjoint): cell
// indices (b = -1 on a PEC wall face), their m0 directions, and v, the mean
// of Ms * m0 before renormalisation to the face Ms.
struct FaceCells {
  long long a, b;
  double ma[3], mb[3], v[3];
};

struct AdjWork;

}  // namespace

// A hard source (Sec. 3.2): its profile dense over the box lo + [0, n).
struct HardSrc {
  int field;              // 0-2: E component, 3-5: H family + 3
  int lo[3], n[3];
  double* d_prof;
  double f0, Tp, t0;
};

struct mm_ctx {
  // geometry
  int nx, ny, nz, per;
  double dx, dy, dz, dt;
  int px, py, pz;
  size_t nelem;
  int prec;
  size_t esz;  // bytes per field element
  double tol;
  int max_iter, fixed_iter;
  int scheme;   // 2: iterative second-order sub-step; 1: first-order (Sec. 3.2.1)
  double H0[3];
  hipStream_t stream;
  void* (*ualloc)(size_t, void*);
  void (*ufree)(void*, void*);
  void* actx;
  size_t dev_bytes;
  std::vector<std::pair<void*, size_t>> allocs;
  std::string err;
  int sticky;  // host copy of the device error word (bits: 1 noconv, 2 nonfinite)

  // fields and cell maps (T = double or float)
  void* E[3];
  void* H[3];
  void* eps;
  void* sig;
  void* mu;
  unsigned char* mat;   // per-cell id into mtab (e_update), or null: dense maps
  void* mtab;           // 256 eps_r then 256 sigma values (T)
  int nmat;

  // magnetic faces
  int nmag;     // evolving faces (families contiguous)
  int nwall;    // magnetic faces on PEC walls (after the evolving ones; frozen)
  int off1, off2;
  std::vector<int> h_idx;  // all magnetic faces: padded index
  std::vector<int> h_fam;
  int* d_idx;
  double *d_Ms, *d_kap, *d_aoms;
  unsigned char* d_fid;       // per evolving face: id of its (Ms, kap, aoms) in d_ftab, or null
  double* d_ftab;             // when at most 256 distinct triples
  int nfmat;
  double* d_M[3];
  double *d_b[3], *d_d[3], *d_q;
  unsigned char* d_nbm;       // neighbour masks of the evolving faces
  void* A[3];                 // shadow H arrays: the H-M iterates rotate through A, B and H
  void* B[3];
  unsigned long long* d_res;  // final iteration count of the two sub-step parities
  unsigned long long* d_part; // residual partials: 2 parities x nres iterations x step_blocks
  int nres;
  unsigned int* d_bar;        // barrier state of hm_finish
  // the control words, partials and barrier state the sub-steps use: the
  // three above, or the fixed device storage during mm_step_noalloc
  unsigned long long* ctl_res;
  unsigned long long* ctl_part;
  unsigned int* ctl_bar;
  void* scratch;              // this device's fixed storage (null if unresolved)
  std::string scratch_err;
  int* ctl_kpred;             // fused form: previous sub-step's iteration count
  unsigned long long* ctl_fpart;  // fused form: partials of hm_fused (2 parities x 4 rows x chunks)

  // fused H-M sub-step (hm_fused.h): chunks of 30 x 6 columns x fL planes
  // holding evolving faces, their slot tables, the second M buffer (Step 1
  // writes it, Step 3 writes d_M back) and the device-side count
  int fuse_mode;              // mm_options.fused
  bool fused_ok;              // the configuration allows the fused form (chunks built)
  bool chain_fused;           // the current run of steps uses it
  int nchunks, fL;
  int* d_forg;
  unsigned* d_fslots;
  double* d_Mb[3];
  unsigned long long* d_fpart;
  int* d_kpred;
  std::vector<unsigned char> h_nbm;
  int step_blocks, fin_blocks;
  int* h_ring;                // pinned: final iteration count of recent sub-steps
  int* d_ring;
  int* d_err;

  // iteration counts: one int per sub-step
  int* d_iters;
  size_t iters_cap;

  // source: dense J0*p over the bounding box of its nonzero interior edges
  int src_comp;
  int nsrc;
  int src_lo[3], src_hi[3];
  double* d_src_prof;
  double f0, Tp, t0;

  // hard sources and surface currents (surface currents become hard H sources)
  std::vector<HardSrc> hard;

  // probes
  std::vector<ProbeRec> probes;
  size_t series_cap;
  double* d_series;
  double* d_sums;
  mmk::PointProbe* d_points;
  int npoints;
  int* d_planes;
  int* d_slots;
  int nflux;
  double* d_partial;
  int flux_blocks;
  void* d_fcap;           // flux-plane capture of the far tiles' fused pass, or null
  unsigned char* d_fmask;  // per plane node: which of its entries the capture holds
  bool fcap_near;          // this step's last near-tile half step fills the capture too
  bool probes_frozen;

  long step;
  int substep;

  // adjoint support (see adjoint_host.h): checkpoints and the iterate log
  double* hlog_cur;           // set while a forward recompute logs iterates
  int hlog_cap;
  bool adj_recompute;         // true while the adjoint recomputes a segment (no probes)
  int ckpt_every;             // 0: adjoint disabled
  int ckpt_inner;             // inner checkpoint spacing of the adjoint (0: single level)
  std::vector<void*> ckpts;   // one device block per checkpoint
  AdjWork* adjw;
  std::vector<FaceCells> fcells;   // per magnetic face (evolving first)
  std::vector<bool> cell_mag;      // Ms > 0 per cell

  // bulk tiles (64 x 4 columns x tkc planes; see mmk::Tiles): every tile,
  // the tiles near evolving magnetic faces (those faces and every face
  // their H_eff reads), and the rest ("far": fused H half steps)
  int tgx, tgy, tgz, tkc;
  int *d_tl_all, *d_tl_near, *d_tl_far;
  int n_all, n_near, n_far;
  unsigned char* d_far;      // per tile id: 1 if far
  std::vector<unsigned char> h_farv;   // the same, on the host
  long long cells_near, cells_far;
  int* d_tl_pml;             // tiles holding open-boundary layer entries
  int n_pml;
  // the E update's list as pairs of tiles stacked in y (lower tile listed;
  // blocks of 64 x 8) and the tiles left unpaired (64 x 4).  (Pairs made
  // h_far slower, 0.442 -> 0.460 ms on the filter grid; it keeps d_tl_far.)
  int *d_tl_all2, *d_tl_all1;
  int n_all2, n_all1;

  // open boundary (split-field PML): per axis damping factors at nodes (E)
  // and cell centres (H), kappa > 0 flags, the stored split parts
  bool has_pml;
  int pml_cells[6];
  double pml_R0, pml_order;
  std::vector<double> pml_kn[3], pml_kc[3];   // kappa at nodes / centres (host)
  double *d_pdn[3], *d_pdc[3];
  unsigned char *d_pon_n[3], *d_pon_c[3];
  void* PE[3];
  void* PH[3];

  // optional kernel timing (mm_profile)
  bool prof;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  std::vector<int> ev_class;
  size_t ev_used;
};

namespace {

mm_status fail(mm_ctx* c, mm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIPCHECK(ctx, call)                                                              \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, MM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

// Fixed device storage for mm_step_noalloc, the entry point for callers
// that cannot allocate: the sub-step control of such a call (two final-count
// words, the barrier state of hm_finish, the residual partials) lives here
// instead of in the context.  Each device holds its own copy until the
// process ends; the host resolves its address once per device at mm_init
// (the array's name in host code is not a device address).
constexpr size_t kScratchHeader = 256;   // [0, 16) final counts, [64, 72) barrier, [128, 132) count
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];

// Bytes of sub-step control one call needs: header plus 2 parities x nres
// iterations x step_blocks partials.
size_t ctl_bytes(const mm_ctx* c) {
  return kScratchHeader + 2 * (size_t)c->nres * (size_t)c->step_blocks * sizeof(unsigned long long) +
         2 * 4 * (size_t)c->nchunks * sizeof(unsigned long long);
}

// Once per device, with that device current: the address of `scratch`.
void resolve_scratch(mm_ctx* c) {
  c->scratch = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    c->scratch_err = e != hipSuccess ? hipGetErrorString(e) : "device ordinal out of range";
    return;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      c->scratch_err = e != hipSuccess ? hipGetErrorString(e) : "null symbol address";
      return;
    }
    g_scratch_addr[dev] = p;
  }
  c->scratch = g_scratch_addr[dev];
}

__global__ void zero_words(unsigned int* p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0u;
}

__global__ void copy_word(int* dst, const int* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

void* dalloc(mm_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (c->ualloc && c->ufree) {
    p = c->ualloc(bytes, c->actx);
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  }
  if (p) {
    c->allocs.push_back({p, bytes});
    c->dev_bytes += bytes;
  }
  return p;
}

void dfree(mm_ctx* c, void* p) {
  if (!p) return;
  for (size_t q = 0; q < c->allocs.size(); ++q) {
    if (c->allocs[q].first == p) {
      c->dev_bytes -= c->allocs[q].second;
      c->allocs.erase(c->allocs.begin() + q);
      break;
    }
  }
  if (c->ualloc && c->ufree) c->ufree(p, c->actx);
  else (void)hipFree(p);
}

inline size_t pidx(const mm_ctx* c, int i, int j, int k) {
  return (size_t)i + (size_t)c->px * ((size_t)j + (size_t)c->py * (size_t)k);
}

inline int nodes(const mm_ctx* c, int ax) {
  const int n = ax == 0 ? c->nx : (ax == 1 ? c->ny : c->nz);
  return (c->per >> ax & 1) ? n : n + 1;
}

inline int ncell(const mm_ctx* c, int ax) { return ax == 0 ? c->nx : (ax == 1 ? c->ny : c->nz); }

// staggered extent of field id 0..5 (E edges, H faces), and 6..17 (faces)
void field_extent(const mm_ctx* c, int field, int ext[3]) {
  if (field < 3) {
    for (int a = 0; a < 3; ++a) ext[a] = (a == field) ? ncell(c, a) : nodes(c, a);
  } else {
    int f;
    if (field < 6) f = field - 3;
    else if (field < 15) f = (field - 6) / 3;
    else f = field - 15;
    for (int a = 0; a < 3; ++a) ext[a] = (a == f) ? nodes(c, a) : ncell(c, a);
  }
}

// is staggered entry (i,j,k) of E/H component `field` (0..5) interior?
bool entry_interior(const mm_ctx* c, int field, int i, int j, int k) {
  const int p[3] = {i, j, k};
  if (field < 3) {
    for (int a = 0; a < 3; ++a) {
      if (a == field || (c->per >> a & 1)) continue;
      if (p[a] == 0 || p[a] == ncell(c, a)) return false;
    }
    return true;
  }
  const int f = field - 3;
  if (c->per >> f & 1) return true;
  return !(p[f] == 0 || p[f] == ncell(c, f));
}

double cell(const double* a, double def, const mm_ctx* c, int i, int j, int k) {
  if (!a) return def;
  return a[(size_t)i + (size_t)c->nx * ((size_t)j + (size_t)c->ny * (size_t)k)];
}

double waveform(double t, double f0, double Tp, double t0) {
  return std::exp(-((t - t0) * (t - t0)) / (2.0 * Tp * Tp)) * std::cos(2.0 * M_PI * f0 * t);
}

template <typename T>
mm_status upload_cellmap(mm_ctx* c, const double* src, double def, void** dst) {
  std::vector<T> h(c->nelem, (T)0);
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) h[pidx(c, i, j, k)] = (T)cell(src, def, c, i, j, k);
  *dst = dalloc(c, c->nelem * sizeof(T));
  if (!*dst) return fail(c, MM_ENOMEM, "device allocation of a cell map failed");
  HIPCHECK(c, hipMemcpy(*dst, h.data(), c->nelem * sizeof(T), hipMemcpyHostToDevice));
  return MM_OK;
}

// Byte material ids for the E update when the grid holds at most 256
// distinct (eps_r, sigma) pairs (after conversion to the storage type, so
// the table holds exactly the values of the dense maps); otherwise none.
template <typename T>
mm_status build_material_ids(mm_ctx* c, const mm_materials* mat) {
  c->mat = nullptr;
  c->mtab = nullptr;
  c->nmat = 0;
  std::vector<unsigned char> ids(c->nelem, 0);
  std::vector<T> tab(512, (T)0);
  std::unordered_map<uint64_t, int> seen;
  auto bits = [](T v) {
    uint64_t b = 0;
    std::memcpy(&b, &v, sizeof(T));
    return b;
  };
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        const T e = (T)cell(mat->eps_r, 1.0, c, i, j, k);
        const T sg = (T)cell(mat->sigma, 0.0, c, i, j, k);
        const uint64_t key = bits(e) * 0x9E3779B97F4A7C15ull ^ bits(sg);
        auto it = seen.find(key);
        int id;
        if (it == seen.end()) {
          id = (int)seen.size();
          if (id >= 256) return MM_OK;   // too many: dense maps
          seen.emplace(key, id);
          tab[id] = e;
          tab[256 + id] = sg;
        } else {
          id = it->second;
          if (bits(tab[id]) != bits(e) || bits(tab[256 + id]) != bits(sg)) return MM_OK;  // key clash: dense
        }
        ids[pidx(c, i, j, k)] = (unsigned char)id;
      }
  c->mat = (unsigned char*)dalloc(c, c->nelem);
  c->mtab = dalloc(c, 512 * sizeof(T));
  if (!c->mat || !c->mtab) return fail(c, MM_ENOMEM, "material-id allocation failed");
  HIPCHECK(c, hipMemcpy(c->mat, ids.data(), c->nelem, hipMemcpyHostToDevice));
  HIPCHECK(c, hipMemcpy(c->mtab, tab.data(), 512 * sizeof(T), hipMemcpyHostToDevice));
  c->nmat = (int)seen.size();
  return MM_OK;
}

mm_status grow_buffers(mm_ctx* c, size_t need_steps) {
  // iteration counts (2 per step) and probe series
  if (2 * need_steps > c->iters_cap) {
    size_t cap = std::max<size_t>(2 * need_steps, 2 * c->iters_cap);
    cap = std::max<size_t>(cap, 1024);
    int* p = (int*)dalloc(c, cap * sizeof(int));
    if (!p) return fail(c, MM_ENOMEM, "allocation of the iteration log failed");
    if (c->d_iters && c->iters_cap)
      HIPCHECK(c, hipMemcpyAsync(p, c->d_iters, c->iters_cap * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    dfree(c, c->d_iters);
    c->d_iters = p;
    c->iters_cap = cap;
  }
  const size_t np = c->probes.size();
  if (np && need_steps > c->series_cap) {
    size_t cap = std::max<size_t>(need_steps, 2 * c->series_cap);
    cap = std::max<size_t>(cap, 256);
    double* p = (double*)dalloc(c, np * cap * sizeof(double));
    if (!p) return fail(c, MM_ENOMEM, "allocation of the probe series failed");
    if (c->d_series && c->series_cap)
      HIPCHECK(c, hipMemcpy2DAsync(p, cap * sizeof(double), c->d_series, c->series_cap * sizeof(double),
                                   c->series_cap * sizeof(double), np, hipMemcpyDeviceToDevice, c->stream));
    dfree(c, c->d_series);
    c->d_series = p;
    c->series_cap = cap;
    // the point descriptors do not depend on the capacity
  }
  return MM_OK;
}

// Which entries of each flux-plane node the capture holds.  Far tiles (the
// fused pass of the far tiles writes them): bit 0 for the node's x = i0
// entries, bit 1 for its x = im entries.  Near tiles (the fused sub-step's
// last half step writes them): bit 2 for E_y, E_z at i0, bits 3 and 4 for
// H_y, H_z at i0, bits 5 and 6 for H_y, H_z at im, each unless that face
// is an evolving magnetic face (its H comes from the iteration).  Only
// entries inside the grid (i < nx, j < ny, k < nz).
mm_status flux_mask(mm_ctx* c) {
  if (!c->d_fmask) return MM_OK;
  const int NY = nodes(c, 1), NZ = nodes(c, 2);
  // evolving faces per family, sorted by padded index
  std::vector<int> ev[3];
  for (int t = 0; t < c->nmag; ++t) ev[c->h_fam[t]].push_back((int)c->h_idx[t]);
  for (auto& v : ev) std::sort(v.begin(), v.end());
  auto evolving = [&](int f, int i, int j, int k) {
    const int pi = (int)pidx(c, i, j, k);
    return std::binary_search(ev[f].begin(), ev[f].end(), pi);
  };
  std::vector<unsigned char> mask((size_t)c->nflux * NY * NZ, 0);
  int p = 0;
  for (const ProbeRec& r : c->probes) {
    if (r.d.kind == 0) continue;
    const int i0 = r.d.i;
    const int im = (c->per & 1) && i0 == 0 ? c->nx - 1 : i0 - 1;
    for (int j = 0; j < NY; ++j)
      for (int k = 0; k < NZ; ++k) {
        auto tile_of = [&](int i) -> int {   // 1 far, 0 near, -1 outside the grid
          if (i < 0 || i >= c->nx || j >= c->ny || k >= c->nz || c->h_farv.empty()) return -1;
          const size_t id = (size_t)(i / 64) + (size_t)c->tgx * ((size_t)(j / 4) + (size_t)c->tgy * (size_t)(k / c->tkc));
          return c->h_farv[id] != 0 ? 1 : 0;
        };
        const int t0 = tile_of(i0), tm = tile_of(im);
        unsigned char m = 0;
        if (t0 == 1) m |= 1;
        if (tm == 1) m |= 2;
        if (t0 == 0) {
          m |= 4;
          if (!evolving(1, i0, j, k)) m |= 8;
          if (!evolving(2, i0, j, k)) m |= 16;
        }
        if (tm == 0) {
          if (!evolving(1, im, j, k)) m |= 32;
          if (!evolving(2, im, j, k)) m |= 64;
        }
        mask[(size_t)p * NY * NZ + (size_t)j * NZ + k] = m;
      }
    ++p;
  }
  HIPCHECK(c, hipMemcpy(c->d_fmask, mask.data(), mask.size(), hipMemcpyHostToDevice));
  return MM_OK;
}

mm_status freeze_probes(mm_ctx* c) {
  if (c->probes_frozen) return MM_OK;
  c->probes_frozen = true;
  const size_t np = c->probes.size();
  if (!np) return MM_OK;
  std::vector<mmk::PointProbe> pts;
  std::vector<int> planes, slots;
  for (size_t s = 0; s < np; ++s) {
    if (c->probes[s].d.kind == 0) {
      mmk::PointProbe q = c->probes[s].pp;
      q.slot = (int)s;
      pts.push_back(q);
    } else {
      planes.push_back(c->probes[s].d.i);
      slots.push_back((int)s);
    }
  }
  c->npoints = (int)pts.size();
  c->nflux = (int)planes.size();
  c->d_sums = (double*)dalloc(c, np * sizeof(double));
  if (!c->d_sums) return fail(c, MM_ENOMEM, "probe allocation failed");
  HIPCHECK(c, hipMemsetAsync(c->d_sums, 0, np * sizeof(double), c->stream));
  if (c->npoints) {
    c->d_points = (mmk::PointProbe*)dalloc(c, pts.size() * sizeof(mmk::PointProbe));
    if (!c->d_points) return fail(c, MM_ENOMEM, "probe allocation failed");
    HIPCHECK(c, hipMemcpy(c->d_points, pts.data(), pts.size() * sizeof(mmk::PointProbe), hipMemcpyHostToDevice));
  }
  if (c->nflux) {
    c->flux_blocks = (nodes(c, 1) * nodes(c, 2) + 255) / 256;   // one thread per node of the plane
    c->d_planes = (int*)dalloc(c, planes.size() * sizeof(int));
    c->d_slots = (int*)dalloc(c, slots.size() * sizeof(int));
    c->d_partial = (double*)dalloc(c, (size_t)c->nflux * 2 * c->flux_blocks * sizeof(double));
    if (!c->d_planes || !c->d_slots || !c->d_partial)
      return fail(c, MM_ENOMEM, "probe allocation failed");
    HIPCHECK(c, hipMemcpy(c->d_planes, planes.data(), planes.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->d_slots, slots.data(), slots.size() * sizeof(int), hipMemcpyHostToDevice));
    // the far tiles' pass stores at most one plane per 64-column tile row
    // and role (x = i0, x = im)
    bool fcap = c->nflux <= mmk::kCapPlanes;
    for (int p = 0; p < c->nflux && fcap; ++p)
      for (int q = 0; q < p; ++q) {
        const int ip = planes[p], iq = planes[q];
        const int mp = (c->per & 1) && ip == 0 ? c->nx - 1 : ip - 1, mq = (c->per & 1) && iq == 0 ? c->nx - 1 : iq - 1;
        if (ip / 64 == iq / 64 || mp / 64 == mq / 64) fcap = false;
      }
    if (fcap) {
      c->d_fcap = dalloc(c, (size_t)c->nflux * 6 * nodes(c, 1) * nodes(c, 2) * c->esz);
      c->d_fmask = (unsigned char*)dalloc(c, (size_t)c->nflux * nodes(c, 1) * nodes(c, 2));
      if (!c->d_fcap || !c->d_fmask) return fail(c, MM_ENOMEM, "probe allocation failed");
      mm_status ms = flux_mask(c);
      if (ms) return ms;
    }
  }
  return MM_OK;
}

// Bracket a launch with an event pair when profiling is on.
struct Timed {
  mm_ctx* c;
  int cls;
  hipEvent_t stop = nullptr;
  Timed(mm_ctx* ctx, int k) : c(ctx), cls(k) {
    if (!c->prof) return;
    if (c->ev_used == c->ev_pool.size()) {
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        c->prof = false;
        return;
      }
      c->ev_pool.push_back({a, b});
      c->ev_class.push_back(0);
    }
    c->ev_class[c->ev_used] = cls;
    (void)hipEventRecord(c->ev_pool[c->ev_used].first, c->stream);
    stop = c->ev_pool[c->ev_used].second;
  }
  ~Timed() {
    if (!stop) return;
    (void)hipEventRecord(stop, c->stream);
    c->ev_used++;
  }
};

Geo make_geo(const mm_ctx* c) {
  Geo g;
  g.nx = c->nx;
  g.ny = c->ny;
  g.nz = c->nz;
  g.px = c->px;
  g.sz = c->px * c->py;
  g.per = c->per;
  g.dx = c->dx;
  g.dy = c->dy;
  g.dz = c->dz;
  g.idx = 1.0 / c->dx;
  g.idy = 1.0 / c->dy;
  g.idz = 1.0 / c->dz;
  return g;
}

template <typename T>
mmk::Fields<T> make_fields(const mm_ctx* c) {
  mmk::Fields<T> F;
  for (int a = 0; a < 3; ++a) {
    F.E[a] = (T*)c->E[a];
    F.H[a] = (T*)c->H[a];
    F.A[a] = (T*)c->A[a];
    F.B[a] = (T*)c->B[a];
  }
  return F;
}

mmk::Mag make_mag(const mm_ctx* c) {
  mmk::Mag m;
  m.idx = c->d_idx;
  m.Ms = c->d_Ms;
  m.kap = c->d_kap;
  m.aoms = c->d_aoms;
  m.fid = c->d_fid;
  m.ftab = c->d_ftab;
  for (int a = 0; a < 3; ++a) {
    m.M[a] = c->d_M[a];
    m.b[a] = c->d_b[a];
    m.d[a] = c->d_d[a];
  }
  m.q = c->d_q;
  m.nbm = c->d_nbm;
  m.hlog = c->hlog_cur;
  m.hlog_cap = c->hlog_cap;
  m.off1 = c->off1;
  m.off2 = c->off2;
  m.n = c->nmag;
  return m;
}

mmk::Tiles tiles(const mm_ctx* c, const int* list, int split = 1) {
  mmk::Tiles t;
  t.list = list;
  t.gx = c->tgx;
  t.gy = c->tgy;
  t.kc = c->tkc;
  t.split = split;
  return t;
}

template <typename T>
mmk::Pml<T> make_pml(const mm_ctx* c) {
  mmk::Pml<T> P;
  for (int a = 0; a < 3; ++a) {
    P.dn[a] = c->d_pdn[a];
    P.dc[a] = c->d_pdc[a];
    P.on_n[a] = c->d_pon_n[a];
    P.on_c[a] = c->d_pon_c[a];
    P.PE[a] = (T*)c->PE[a];
    P.PH[a] = (T*)c->PH[a];
  }
  return P;
}

// z-split for a launch over n tiles: enough blocks to fill the chip
// (~4096 blocks, 16 waves per CU), runs of at least 4 planes.
int split_for(const mm_ctx* c, int n) {
  if (n <= 0) return 1;
  const int want = (4096 + n - 1) / n;
  return std::max(1, std::min(want, c->tkc / 4));
}

int kchunk_for(const mm_ctx* c, dim3& grid) {
  const int gx = (c->nx + 63) / 64, gy = (c->ny + 3) / 4;
  // aim for >= ~4096 blocks while keeping each z run long enough to reuse
  // the carried plane
  int chunks = std::max(1, 4096 / std::max(1, gx * gy));
  int kc = std::max(4, (c->nz + chunks - 1) / chunks);
  kc = std::min(kc, c->nz);
  grid = dim3(gx, gy, (c->nz + kc - 1) / kc);
  return kc;
}

// Number of iterations to enqueue as ordinary launches: one more than the
// largest count seen in the last 64 sub-steps (read from pinned memory the
// device writes; stale values are harmless because hm_finish completes any
// iterations that were not enqueued).  The spare launch usually only finds
// that the stopping rule has fired, at no measurable cost; when the count
// rises by one it runs that iteration on the full grid instead of on
// hm_finish's small co-resident one.
int iterations_to_enqueue(const mm_ctx* c) {
  if (c->fixed_iter > 0) return c->fixed_iter;
  int mx = 1;
  for (int q = 0; q < 64; ++q) mx = std::max(mx, (int)((volatile int*)c->h_ring)[q]);
  return std::max(1, std::min(std::min(mx + 1, 32), c->max_iter));
}

// Hard sources on E (e_field) or H, value g(t).
template <typename T>
mm_status apply_hard(mm_ctx* c, bool e_field, double t) {
  for (const HardSrc& hs : c->hard) {
    if ((hs.field < 3) != e_field) continue;
    mmk::Hard k;
    k.prof = hs.d_prof;
    for (int a = 0; a < 3; ++a) {
      k.lo[a] = hs.lo[a];
      k.n[a] = hs.n[a];
    }
    k.comp = hs.field;
    k.g = waveform(t, hs.f0, hs.Tp, hs.t0);
    T* f = (T*)(hs.field < 3 ? c->E[hs.field] : c->H[hs.field - 3]);
    const long long nb = (long long)hs.n[0] * hs.n[1] * hs.n[2];
    hipLaunchKernelGGL((mmk::hard_set<T>), dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, c->stream,
                       make_geo(c), f, k);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// The fused form of one H-M sub-step (hm_fused.h).  Within a run of steps
// the near tiles' H alternates between H (Step 1 writes it, so the E update
// reads it) and the shadow A (Step 3 writes it), M between d_M (Step 3) and
// d_Mb (Step 1); the far tiles stay in H.  run_steps copies the near tiles
// H -> A when a run starts and A -> H when it ends.
template <typename T>
mmk::FluxCap<T> flux_cap(const mm_ctx* c, bool on);

template <typename T>
mm_status substep_fused(mm_ctx* c, bool near_only, bool step3) {
  const Geo g = make_geo(c);
  const double h = 0.5 * c->dt;
  const double hmu0 = h / mmk::kMu0;
  T* X[3];
  T* Y[3];
  for (int a = 0; a < 3; ++a) {
    X[a] = (T*)c->H[a];
    Y[a] = (T*)c->A[a];
  }
  T** Hin = step3 ? X : Y;
  T** Hout = step3 ? Y : X;
  double** Min = step3 ? c->d_Mb : c->d_M;
  double** Mout = step3 ? c->d_M : c->d_Mb;
  if (c->n_near > 0) {
    const int split = split_for(c, c->n_near);
    const mmk::Tiles tl = tiles(c, c->d_tl_near, split);
    const mmk::FluxCap<T> fc = flux_cap<T>(c, step3 && c->fcap_near);
    Timed tm(c, 1);
#define MM_HDB(MU)                                                                                           \
  hipLaunchKernelGGL((mmk::h_half_db<T, MU>), dim3(c->n_near * split), dim3(64, 4), 0, c->stream, g, Hin[0], \
                     Hin[1], Hin[2], Hout[0], Hout[1], Hout[2], (const T*)c->E[0], (const T*)c->E[1],        \
                     (const T*)c->E[2], (const T*)c->mu, (T)hmu0, (T)h, tl, fc)
    if (c->mu) MM_HDB(true);
    else MM_HDB(false);
#undef MM_HDB
  }
  if (!near_only && c->n_far > 0) {
    const int split = split_for(c, c->n_far);
    const mmk::Tiles tl = tiles(c, c->d_tl_far, split);
    Timed tm(c, 1);
#define MM_HFAR1(MU)                                                                                          \
  hipLaunchKernelGGL((mmk::h_bulk<T, MU, 1>), dim3(c->n_far * split), dim3(64, 4), 0, c->stream, g, X[0],      \
                     X[1], X[2], (const T*)c->E[0], (const T*)c->E[1], (const T*)c->E[2], (const T*)c->mu,    \
                     (T)hmu0, (T)h, tl)
    if (c->mu) MM_HFAR1(true);
    else MM_HFAR1(false);
#undef MM_HFAR1
  }
  HIPCHECK(c, hipGetLastError());
  mmk::Mag m = make_mag(c);
  m.hlog = nullptr;
  m.hlog_cap = 0;
  unsigned long long* fpart = c->ctl_fpart + (size_t)(c->substep & 1) * 4 * c->nchunks;
  {
    mmk::FusedArgs<T> a;
    for (int q = 0; q < 3; ++q) {
      a.Hin[q] = Hin[q];
      a.Hout[q] = Hout[q];
      a.E[q] = (const T*)c->E[q];
      a.Min[q] = Min[q];
      a.Mout[q] = Mout[q];
    }
    a.slots = c->d_fslots;
    a.org = c->d_forg;
    a.L = c->fL;
    a.nfmat = c->nfmat;
    a.kfix = c->fixed_iter;
    a.kpred = c->ctl_kpred;
    a.m = m;
    a.H0x = c->H0[0];
    a.H0y = c->H0[1];
    a.H0z = c->H0[2];
    a.hmu0 = hmu0;
    a.part = fpart;
    a.P = c->nchunks;
    Timed tm(c, 2);
    hipLaunchKernelGGL((mmk::hm_fused<T>), dim3(c->nchunks), dim3(mmk::kFCols), 0, c->stream, g, a);
  }
  HIPCHECK(c, hipGetLastError());
  {
    mmk::MoreArgs<T> b;
    for (int q = 0; q < 3; ++q) {
      b.Hin[q] = Hin[q];
      b.Hout[q] = Hout[q];
      b.S[q] = (T*)c->B[q];
      b.E[q] = (const T*)c->E[q];
      b.Min[q] = Min[q];
      m.M[q] = Mout[q];
    }
    b.m = m;
    b.H0x = c->H0[0];
    b.H0y = c->H0[1];
    b.H0z = c->H0[2];
    b.hmu0 = hmu0;
    b.fpart = fpart;
    b.Pf = c->nchunks;
    b.kfix = c->fixed_iter;
    b.kpred = c->ctl_kpred;
    mmk::Ctl C;
    C.cur = c->ctl_res + (c->substep & 1);
    C.next = c->ctl_res + ((c->substep + 1) & 1);
    C.P = c->step_blocks;
    C.part = c->ctl_part + (size_t)(c->substep & 1) * c->nres * c->step_blocks;
    C.tol = c->tol;
    C.max_iter = c->max_iter;
    C.fixed_iter = c->fixed_iter;
    Timed tm(c, 3);
    hipLaunchKernelGGL((mmk::hm_more<T>), dim3(c->fin_blocks), dim3(256), 0, c->stream, g, b, C,
                       c->d_iters + c->substep, c->d_ring + (c->substep & 63), c->ctl_bar, c->d_err);
  }
  HIPCHECK(c, hipGetLastError());
  c->substep++;
  return MM_OK;
}

// One H-M sub-step (Step 1, or Step 3 when step3).  near_only: the Faraday
// half step runs on the near tiles only (the far tiles take it inside the
// fused pass of h_far).
template <typename T>
mm_status substep(mm_ctx* c, bool near_only = false, bool step3 = false) {
  if (c->chain_fused) return substep_fused<T>(c, near_only, step3);
  Geo g = make_geo(c);
  mmk::Fields<T> F = make_fields<T>(c);
  const double h = 0.5 * c->dt;
  const double hmu0 = h / mmk::kMu0;
  mmk::Ctl C;
  C.cur = c->ctl_res + (c->substep & 1);
  C.next = c->ctl_res + ((c->substep + 1) & 1);
  C.P = c->step_blocks;
  C.part = c->ctl_part + (size_t)(c->substep & 1) * c->nres * c->step_blocks;
  C.tol = c->tol;
  C.max_iter = c->max_iter;
  C.fixed_iter = c->fixed_iter;
  const double H0x = c->H0[0], H0y = c->H0[1], H0z = c->H0[2];
  if (c->nmag > 0) {
    mmk::Mag m = make_mag(c);
    Timed tm(c, 2);
    hipLaunchKernelGGL((mmk::hm_pre<T>), dim3(c->step_blocks), dim3(MM_MAG_THREADS), 0, c->stream, g, F, m, h, hmu0,
                       H0x, H0y, H0z, c->scheme == 1 ? 1 : 0, C, c->d_err);
  }
  HIPCHECK(c, hipGetLastError());
  const int nt = near_only ? c->n_near : c->n_all;
  if (nt > 0) {
    const int split = split_for(c, nt);
    const mmk::Tiles tl = tiles(c, near_only ? c->d_tl_near : c->d_tl_all, split);
    Timed tm(c, 1);
    if (c->mu)
      hipLaunchKernelGGL((mmk::h_bulk<T, true, 1>), dim3(nt * split), dim3(64, 4), 0, c->stream, g, (T*)c->H[0],
                         (T*)c->H[1], (T*)c->H[2], (const T*)c->E[0], (const T*)c->E[1], (const T*)c->E[2],
                         (const T*)c->mu, (T)hmu0, (T)h, tl);
    else
      hipLaunchKernelGGL((mmk::h_bulk<T, false, 1>), dim3(nt * split), dim3(64, 4), 0, c->stream, g, (T*)c->H[0],
                         (T*)c->H[1], (T*)c->H[2], (const T*)c->E[0], (const T*)c->E[1], (const T*)c->E[2],
                         (const T*)c->mu, (T)hmu0, (T)h, tl);
  }
  if (c->n_pml > 0) {
    const int split = split_for(c, c->n_pml);
    const mmk::Tiles tl = tiles(c, c->d_tl_pml, split);
    const mmk::Pml<T> P = make_pml<T>(c);
    Timed tm(c, 1);
    if (c->mu)
      hipLaunchKernelGGL((mmk::pml_h<T, true>), dim3(c->n_pml * split), dim3(64, 4), 0, c->stream, g,
                         (T*)c->H[0], (T*)c->H[1], (T*)c->H[2], (const T*)c->E[0], (const T*)c->E[1],
                         (const T*)c->E[2], (const T*)c->mu, (T)hmu0, (T)h, tl, P);
    else
      hipLaunchKernelGGL((mmk::pml_h<T, false>), dim3(c->n_pml * split), dim3(64, 4), 0, c->stream, g,
                         (T*)c->H[0], (T*)c->H[1], (T*)c->H[2], (const T*)c->E[0], (const T*)c->E[1],
                         (const T*)c->E[2], (const T*)c->mu, (T)hmu0, (T)h, tl, P);
  }
  HIPCHECK(c, hipGetLastError());
  if (!c->hard.empty()) {
    mm_status hs = apply_hard<T>(c, false, ((double)c->step + (step3 ? 1.0 : 0.5)) * c->dt);
    if (hs) return hs;
  }
  if (c->nmag > 0) {
    mmk::Mag m = make_mag(c);
    const int R = iterations_to_enqueue(c);
    for (int r = 2; r <= R; ++r) {
      Timed tm(c, 3);
      hipLaunchKernelGGL((mmk::hm_step<T>), dim3(c->step_blocks), dim3(MM_MAG_THREADS), 0, c->stream, g, F, m, H0x, H0y,
                         H0z, C, r, c->d_err);
    }
    HIPCHECK(c, hipGetLastError());
    {
      Timed tm(c, 4);
      hipLaunchKernelGGL((mmk::hm_finish<T>), dim3(c->fin_blocks), dim3(256), 0, c->stream, g, F, m, H0x, H0y,
                         H0z, C, R + 1, c->ctl_bar, c->d_err);
    }
    {
      Timed tm(c, 6);
      hipLaunchKernelGGL((mmk::hm_commit<T>), dim3(c->step_blocks), dim3(MM_MAG_THREADS), 0, c->stream, F, m, C,
                         c->d_iters + c->substep, c->d_ring + (c->substep & 63), c->d_err);
    }
    HIPCHECK(c, hipGetLastError());
  }
  c->substep++;
  return MM_OK;
}

mmk::Src make_src(const mm_ctx* c) {
  mmk::Src src;
  std::memset(&src, 0, sizeof src);
  src.comp = -1;
  if (c->nsrc > 0) {
    src.prof = c->d_src_prof;
    src.comp = c->src_comp;
    for (int a = 0; a < 3; ++a) {
      src.lo[a] = c->src_lo[a];
      src.hi[a] = c->src_hi[a];
    }
    src.g = waveform(((double)c->step + 0.5) * c->dt, c->f0, c->Tp, c->t0);
  }
  return src;
}

// Step 2 of step c->step.  With eout (the adjoint's recompute only; no
// open boundary, no hard sources): E^{n+1} goes to eout, E keeps E^n.
template <typename T>
mm_status e_step(mm_ctx* c, void* const* eout = nullptr) {
  const Geo g = make_geo(c);
  const mmk::Src src = make_src(c);
  Timed tm(c, 0);
  if (eout && (c->n_pml > 0 || !c->hard.empty()))
    return fail(c, MM_ESTATE, "an out-of-place E update needs no open boundary and no hard source");
#define MM_EUPD1(SIG, MAT, RY, N, LIST)                                                                        \
  do {                                                                                                         \
    if (eout)                                                                                                  \
      hipLaunchKernelGGL((mmk::e_update<T, SIG, MAT, RY, true>), dim3(N), dim3(64, RY), 0, c->stream, g,       \
                         (T*)c->E[0], (T*)c->E[1], (T*)c->E[2], (const T*)c->H[0], (const T*)c->H[1],          \
                         (const T*)c->H[2], (const T*)c->eps, (const T*)c->sig, c->mat, (const T*)c->mtab,      \
                         (T)c->dt, src, tiles(c, LIST), (T*)eout[0], (T*)eout[1], (T*)eout[2]);                \
    else                                                                                                       \
      hipLaunchKernelGGL((mmk::e_update<T, SIG, MAT, RY>), dim3(N), dim3(64, RY), 0, c->stream, g,             \
                         (T*)c->E[0], (T*)c->E[1], (T*)c->E[2], (const T*)c->H[0], (const T*)c->H[1],          \
                         (const T*)c->H[2], (const T*)c->eps, (const T*)c->sig, c->mat, (const T*)c->mtab,      \
                         (T)c->dt, src, tiles(c, LIST), (T*)nullptr, (T*)nullptr, (T*)nullptr);                \
  } while (0)
#define MM_EUPD(SIG, MAT)                                                                                      \
  do {                                                                                                         \
    if (c->n_all2 > 0) MM_EUPD1(SIG, MAT, 8, c->n_all2, c->d_tl_all2);                                         \
    if (c->n_all1 > 0) MM_EUPD1(SIG, MAT, 4, c->n_all1, c->d_tl_all1);                                         \
  } while (0)
  if (c->n_all == 0) {
  } else if (c->mat) {
    if (c->sig) MM_EUPD(true, true);
    else MM_EUPD(false, true);
  } else {
    if (c->sig) MM_EUPD(true, false);
    else MM_EUPD(false, false);
  }
#undef MM_EUPD
#undef MM_EUPD1
  if (c->n_pml > 0) {
    const int split = split_for(c, c->n_pml);
    const mmk::Tiles tp = tiles(c, c->d_tl_pml, split);
    const mmk::Pml<T> P = make_pml<T>(c);
    if (c->sig)
      hipLaunchKernelGGL((mmk::pml_e<T, true>), dim3(c->n_pml * split), dim3(64, 4), 0, c->stream, g,
                         (T*)c->E[0], (T*)c->E[1], (T*)c->E[2], (const T*)c->H[0], (const T*)c->H[1],
                         (const T*)c->H[2], (const T*)c->eps, (const T*)c->sig, (T)c->dt, src, tp, P);
    else
      hipLaunchKernelGGL((mmk::pml_e<T, false>), dim3(c->n_pml * split), dim3(64, 4), 0, c->stream, g,
                         (T*)c->E[0], (T*)c->E[1], (T*)c->E[2], (const T*)c->H[0], (const T*)c->H[1],
                         (const T*)c->H[2], (const T*)c->eps, (const T*)c->sig, (T)c->dt, src, tp, P);
  }
  HIPCHECK(c, hipGetLastError());
  if (!c->hard.empty()) return apply_hard<T>(c, true, ((double)c->step + 1.0) * c->dt);
  return MM_OK;
}

// The fused Faraday pass of the far tiles: Step 3 of step n and Step 1 of
// step n+1 (both with curl E^{n+1}), H^{n+1/2} -> H^{n+3/2}.
// The capture descriptor of the flux planes (buf null: none).
template <typename T>
mmk::FluxCap<T> flux_cap(const mm_ctx* c, bool on) {
  mmk::FluxCap<T> fc{};
  if (!on) return fc;
  std::vector<int> planes;
  for (const ProbeRec& r : c->probes)
    if (r.d.kind != 0) planes.push_back(r.d.i);
  fc.buf = (T*)c->d_fcap;
  fc.n = (int)planes.size();
  for (int p = 0; p < fc.n; ++p) {
    fc.i0[p] = planes[p];
    fc.im[p] = (c->per & 1) && planes[p] == 0 ? c->nx - 1 : planes[p] - 1;
  }
  fc.NZ = nodes(c, 2);
  fc.nn = (long long)nodes(c, 1) * fc.NZ;
  return fc;
}

// Whether the far tiles' fused pass stores the flux planes' values (the flux
// probe then runs after it).
bool flux_captured(const mm_ctx* c) {
  return c->d_fcap && c->n_far > 0 && c->tkc <= mmk::kCapPlanesZ && !c->adj_recompute;
}

template <typename T>
mm_status h_far(mm_ctx* c, bool cap = false) {
  if (c->n_far == 0) return MM_OK;
  const Geo g = make_geo(c);
  const mmk::Tiles tl = tiles(c, c->d_tl_far);
  const double h = 0.5 * c->dt, hmu0 = h / mmk::kMu0;
  const mmk::FluxCap<T> fc = flux_cap<T>(c, cap);
  Timed tm(c, 7);
  if (c->mu)
    hipLaunchKernelGGL((mmk::h_bulk<T, true, 2>), dim3(c->n_far), dim3(64, 4), 0, c->stream, g, (T*)c->H[0],
                       (T*)c->H[1], (T*)c->H[2], (const T*)c->E[0], (const T*)c->E[1], (const T*)c->E[2],
                       (const T*)c->mu, (T)hmu0, (T)h, tl, fc);
  else
    hipLaunchKernelGGL((mmk::h_bulk<T, false, 2>), dim3(c->n_far), dim3(64, 4), 0, c->stream, g, (T*)c->H[0],
                       (T*)c->H[1], (T*)c->H[2], (const T*)c->E[0], (const T*)c->E[1], (const T*)c->E[2],
                       (const T*)c->mu, (T)hmu0, (T)h, tl, fc);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// Probe sampling at level c->step + 1.
// lagged: the far tiles hold H^{n+1/2} (the fused pass comes after).
// which: 1 point probes, 2 flux planes, 3 both.  captured: the far tiles'
// fused pass has run with the flux-plane capture (the flux planes only).
template <typename T>
mm_status record_probes(mm_ctx* c, bool lagged = false, int which = 3, bool captured = false) {
  if (c->adj_recompute) return MM_OK;
  const Geo g = make_geo(c);
  const mmk::Fields<T> F = make_fields<T>(c);
  mmk::Lag<T> L;
  L.far = (lagged && c->n_far > 0) ? c->d_far : nullptr;
  for (int a = 0; a < 3; ++a) L.Hn[a] = (lagged && c->chain_fused) ? (const T*)c->A[a] : nullptr;
  L.mu = (const T*)c->mu;
  L.h = (T)(0.5 * c->dt);
  L.coef0 = (T)(0.5 * c->dt / mmk::kMu0);
  L.gx = c->tgx;
  L.gy = c->tgy;
  L.kc = c->tkc;
  if (!(which & 1 ? c->npoints : 0) && !(which & 2 ? c->nflux : 0)) return MM_OK;
  Timed tm(c, 5);
  if ((which & 1) && c->npoints)
    hipLaunchKernelGGL((mmk::probe_points<T>), dim3((c->npoints + 63) / 64), dim3(64), 0, c->stream, g, F, L,
                       c->d_points, c->npoints, c->d_series, c->series_cap, c->d_sums, c->step, c->dt);
  if ((which & 2) && c->nflux) {
    const int NY = nodes(c, 1), NZ = nodes(c, 2);
    hipLaunchKernelGGL((mmk::probe_flux<T>), dim3(c->flux_blocks, c->nflux), dim3(256), 0, c->stream, g, F, L,
                       c->d_planes, c->d_partial, NY, NZ, flux_cap<T>(c, captured), c->d_fmask,
                       (int)(captured && c->fcap_near));
    hipLaunchKernelGGL(mmk::probe_flux_sum, dim3(c->nflux), dim3(256), 0, c->stream, c->d_partial,
                       c->flux_blocks, c->d_slots, c->d_series, c->series_cap, c->d_sums, c->step, c->dt,
                       c->dy * c->dz);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

template <typename T>
mm_status one_step(mm_ctx* c) {
  mm_status s = substep<T>(c);              // Step 1
  if (s) return s;
  s = e_step<T>(c);                         // Step 2
  if (s) return s;
  s = substep<T>(c, false, true);           // Step 3
  if (s) return s;
  s = record_probes<T>(c);
  if (s) return s;
  c->step++;
  return MM_OK;
}

mm_status save_checkpoint(mm_ctx* c, size_t idx);

// n steps with the far tiles' half steps fused across step boundaries.
// Step q starts a chain when the far tiles are at an integer level (first
// step of the call) and ends one when it must leave them there (last step,
// or a checkpoint before the next step); inside a chain the far tiles skip
// Step 1 and Step 3 and take the fused pass after the probes instead.
// Copy the near tiles' H between the field arrays and the shadow A (the
// fused form's second buffer).
template <typename T>
mm_status copy_near(mm_ctx* c, bool to_shadow) {
  if (c->n_near == 0) return MM_OK;
  const Geo g = make_geo(c);
  const int split = split_for(c, c->n_near);
  const mmk::Tiles tl = tiles(c, c->d_tl_near, split);
  void* const* src = to_shadow ? c->H : c->A;
  void* const* dst = to_shadow ? c->A : c->H;
  hipLaunchKernelGGL((mmk::copy_tiles<T>), dim3(c->n_near * split), dim3(64, 4), 0, c->stream, g,
                     (const T*)src[0], (const T*)src[1], (const T*)src[2], (T*)dst[0], (T*)dst[1], (T*)dst[2], tl);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// Whether the next run of steps takes the fused sub-step.
bool fused_for_chain(const mm_ctx* c) {
  // (the adjoint's first recompute, which logs no iterates, may take it)
  if (!c->fused_ok || c->hlog_cur) return false;
  if (c->fixed_iter > mmk::kFMaxK) return false;
  for (const HardSrc& hs : c->hard)
    if (hs.field >= 3) return false;
  return true;
}

template <typename T>
mm_status run_steps(mm_ctx* c, int64_t n) {
  mm_status s;
  bool lagging = false;   // far tiles hold H^{n+1/2} of the current step
  for (int64_t q = 0; q < n; ++q) {
    if (c->ckpt_every > 0 && c->step % c->ckpt_every == 0) {
      s = save_checkpoint(c, (size_t)(c->step / c->ckpt_every));
      if (s) return s;
    }
    const bool end = q == n - 1 || (c->ckpt_every > 0 && (c->step + 1) % c->ckpt_every == 0);
    if (!lagging) {   // a run starts: every tile at level n, everything in H
      c->chain_fused = fused_for_chain(c);
      if (c->chain_fused && (s = copy_near<T>(c, true))) return s;
    }
    if ((s = substep<T>(c, lagging))) return s;     // Step 1
    if ((s = e_step<T>(c))) return s;               // Step 2
    // the flux probe of a lagging step reads the near tiles' plane nodes from
    // the capture as well when the fused sub-step's last half step fills it
    c->fcap_near = !end && c->nflux && c->chain_fused && flux_captured(c);
    s = substep<T>(c, !end, true);                  // Step 3
    c->fcap_near = c->fcap_near && !s;
    if (s) return s;
    if (end && c->chain_fused) {
      if ((s = copy_near<T>(c, false))) return s;
      c->chain_fused = false;
    }
    const bool cap = !end && c->nflux && flux_captured(c);
    if ((s = record_probes<T>(c, !end, cap ? 1 : 3))) return s;
    if (!end && (s = h_far<T>(c, cap))) return s;
    if (cap && (s = record_probes<T>(c, true, 2, true))) return s;
    c->fcap_near = false;
    lagging = !end;
    c->step++;
  }
  return MM_OK;
}

mm_status read_sticky(mm_ctx* c) {
  int w = 0;
  HIPCHECK(c, hipMemcpy(&w, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (w) {
    c->sticky |= w;
    HIPCHECK(c, hipMemset(c->d_err, 0, sizeof(int)));
  }
  return MM_OK;
}

mm_status take_sticky(mm_ctx* c) {
  const int w = c->sticky;
  c->sticky = 0;
  if (w & 4) {
    (void)hipMemset(c->d_bar, 0, 2 * sizeof(unsigned int));
    return fail(c, MM_EDEVICE, "the sub-step completion barrier timed out");
  }
  if (w & 2) return fail(c, MM_ENONFINITE, "a sub-step residual was not finite");
  if (w & 1) return fail(c, MM_ENOCONV, "a sub-step reached max_iter without meeting tol");
  return MM_OK;
}

bool finite_nonneg(const double* a, size_t n, bool strictly_positive) {
  if (!a) return true;
  for (size_t q = 0; q < n; ++q) {
    if (!std::isfinite(a[q])) return false;
    if (strictly_positive ? !(a[q] > 0) : !(a[q] >= 0)) return false;
  }
  return true;
}

// Open boundary: damping rate kappa per axis at the nodes and the cell
// centres, kappa = kappa_max (depth / thickness)^order inside a layer
// (depth in cells from its inner face), kappa_max = -(order + 1) c ln(R0) /
// (2 thickness); both layers of an axis add.
mm_status setup_pml(mm_ctx* c, const mm_pml* p) {
  c->has_pml = false;
  for (int a = 0; a < 6; ++a) c->pml_cells[a] = 0;
  if (!p) return MM_OK;
  const int n3[3] = {c->nx, c->ny, c->nz};
  const double d3[3] = {c->dx, c->dy, c->dz};
  for (int a = 0; a < 3; ++a) {
    const int lo = p->cells[2 * a], hi = p->cells[2 * a + 1];
    if (lo < 0 || hi < 0 || lo + hi >= n3[a]) return fail(c, MM_EINVAL, "bad PML thickness on axis %d", a);
    if ((lo || hi) && (c->per >> a & 1)) return fail(c, MM_EINVAL, "a PML needs a PEC axis (axis %d is periodic)", a);
    c->pml_cells[2 * a] = lo;
    c->pml_cells[2 * a + 1] = hi;
    if (lo || hi) c->has_pml = true;
  }
  if (!c->has_pml) return MM_OK;
  if (!(p->R0 > 0 && p->R0 < 1) || !(p->order >= 1)) return fail(c, MM_EINVAL, "bad PML grading (R0, order)");
  c->pml_R0 = p->R0;
  c->pml_order = p->order;
  for (int a = 0; a < 3; ++a) {
    const int n = n3[a];
    std::vector<double>& kn = c->pml_kn[a];
    std::vector<double>& kc = c->pml_kc[a];
    kn.assign(n + 1, 0.0);
    kc.assign(n, 0.0);
    for (int side = 0; side < 2; ++side) {
      const int thick = c->pml_cells[2 * a + side];
      if (thick <= 0) continue;
      const double L = thick * d3[a];
      const double kmax = -(p->order + 1) * kC0 * std::log(p->R0) / (2.0 * L);
      for (int q = 0; q <= n; ++q) {
        const double depth = side == 0 ? (double)thick - q : q - (double)(n - thick);
        if (depth > 0) kn[q] += kmax * std::pow(depth / thick, p->order);
      }
      for (int q = 0; q < n; ++q) {
        const double depth = side == 0 ? (double)thick - (q + 0.5) : (q + 0.5) - (double)(n - thick);
        if (depth > 0) kc[q] += kmax * std::pow(depth / thick, p->order);
      }
    }
  }
  return MM_OK;
}

// Device copies of the layer data and the split-part arrays; magnetic
// faces with layer damping are rejected.
mm_status upload_pml(mm_ctx* c) {
  if (!c->has_pml) return MM_OK;
  static const int PMa[3][2] = {{1, 2}, {2, 0}, {0, 1}};
  for (size_t t = 0; t < c->h_idx.size(); ++t) {
    const int pi = c->h_idx[t], f = c->h_fam[t];
    const int k = pi / (c->px * c->py), rr = pi - k * c->px * c->py, j = rr / c->px, i = rr - j * c->px;
    const int q[3] = {i, j, k};
    const int p = PMa[f][0], m = PMa[f][1];
    if (c->pml_kc[p][q[p]] > 0 || c->pml_kc[m][q[m]] > 0)
      return fail(c, MM_EINVAL, "magnetic faces inside the PML are not supported (Sec. 3.2.3)");
  }
  for (int a = 0; a < 3; ++a) {
    const std::vector<double>& kn = c->pml_kn[a];
    const std::vector<double>& kc = c->pml_kc[a];
    std::vector<double> dn(kn.size()), dc(kc.size());
    std::vector<unsigned char> on(kn.size()), oc(kc.size());
    for (size_t q = 0; q < kn.size(); ++q) {
      dn[q] = std::exp(-kn[q] * c->dt / 2.0);
      on[q] = kn[q] > 0;
    }
    for (size_t q = 0; q < kc.size(); ++q) {
      dc[q] = std::exp(-kc[q] * c->dt / 4.0);
      oc[q] = kc[q] > 0;
    }
    c->d_pdn[a] = (double*)dalloc(c, dn.size() * 8);
    c->d_pdc[a] = (double*)dalloc(c, dc.size() * 8);
    c->d_pon_n[a] = (unsigned char*)dalloc(c, on.size());
    c->d_pon_c[a] = (unsigned char*)dalloc(c, oc.size());
    c->PE[a] = dalloc(c, c->nelem * c->esz);
    c->PH[a] = dalloc(c, c->nelem * c->esz);
    if (!c->d_pdn[a] || !c->d_pdc[a] || !c->d_pon_n[a] || !c->d_pon_c[a] || !c->PE[a] || !c->PH[a])
      return fail(c, MM_ENOMEM, "PML allocation failed");
    HIPCHECK(c, hipMemcpy(c->d_pdn[a], dn.data(), dn.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->d_pdc[a], dc.data(), dc.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->d_pon_n[a], on.data(), on.size(), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->d_pon_c[a], oc.data(), oc.size(), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemset(c->PE[a], 0, c->nelem * c->esz));
    HIPCHECK(c, hipMemset(c->PH[a], 0, c->nelem * c->esz));
  }
  return MM_OK;
}

// Launch order of a set of tiles: the dispatcher sends block b to XCD
// b mod 8, so the tiles (in natural order, x fastest) are cut into 8 runs
// of near-equal length and the runs interleaved; each XCD then works on a
// compact slab and the x and y halos its blocks share stay in its L2.
std::vector<int> xcd_order(const std::vector<int>& nat) {
  const size_t n = nat.size(), P = (n + 7) / 8;
  std::vector<int> out;
  out.reserve(n);
  for (size_t q = 0; q < P; ++q)
    for (size_t x = 0; x < 8; ++x) {
      const size_t at = x * P + q;
      if (at < std::min(n, (x + 1) * P)) out.push_back(nat[at]);
    }
  return out;
}

// Tile grid of the bulk kernels and its near/far split.  A tile is near
// when it holds an evolving magnetic face or a face that such a face's
// H_eff reads (all within one cell of it, wrapped on periodic axes).
// At least ~4096 tiles, and no tile deeper than 32 planes: on a grid with a
// wide x-y cross-section deeper tiles give few, long blocks whose last round
// leaves part of the chip idle (1024x512x512 in FP32: 4.99 ms per step with
// 256-plane tiles, 4.51 ms with 32), and coarser near tiles.
mm_status build_tiles(mm_ctx* c) {
  c->tgx = (c->nx + 63) / 64;
  c->tgy = (c->ny + 3) / 4;
  const int chunks = std::max(1, 4096 / std::max(1, c->tgx * c->tgy));
  c->tkc = std::min(std::min(std::max(4, (c->nz + chunks - 1) / chunks), c->nz), 32);
  c->tgz = (c->nz + c->tkc - 1) / c->tkc;
  const size_t nt = (size_t)c->tgx * c->tgy * c->tgz;
  std::vector<unsigned char> near(nt, 0);
  const int n3[3] = {c->nx, c->ny, c->nz};
  for (size_t t = 0; t < (size_t)c->nmag; ++t) {
    const int pi = c->h_idx[t];
    const int k = pi / (c->px * c->py), rr = pi - k * c->px * c->py, j = rr / c->px, i = rr - j * c->px;
    const int p0[3] = {i, j, k};
    for (int dk = -1; dk <= 1; ++dk)
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          int q[3] = {p0[0] + di, p0[1] + dj, p0[2] + dk};
          bool ok = true;
          for (int a = 0; a < 3; ++a) {
            if (c->per >> a & 1) q[a] = (q[a] + n3[a]) % n3[a];
            else if (q[a] < 0 || q[a] >= n3[a]) ok = false;
          }
          if (ok) near[(q[0] / 64) + (size_t)c->tgx * ((q[1] / 4) + (size_t)c->tgy * (q[2] / c->tkc))] = 1;
        }
  }
  // tiles holding a hard H source's faces take every half step on their own
  for (const HardSrc& hs : c->hard) {
    if (hs.field < 3) continue;
    for (int k = hs.lo[2]; k < hs.lo[2] + hs.n[2]; ++k)
      for (int j = hs.lo[1]; j < hs.lo[1] + hs.n[1]; ++j)
        for (int i = hs.lo[0]; i < hs.lo[0] + hs.n[0]; ++i) {
          // a face index along its normal runs to n (the wall); clip to the last cell
          const int q0 = std::min(i, n3[0] - 1), q1 = std::min(j, n3[1] - 1), q2 = std::min(k, n3[2] - 1);
          near[(q0 / 64) + (size_t)c->tgx * ((q1 / 4) + (size_t)c->tgy * (q2 / c->tkc))] = 1;
        }
  }
  // tiles holding layer entries: a cell within one cell of a layer
  std::vector<unsigned char> pmlt(nt, 0);
  if (c->has_pml) {
    auto band = [&](int a, int q) {
      const int lo = c->pml_cells[2 * a], hi = c->pml_cells[2 * a + 1];
      return (lo > 0 && q <= lo) || (hi > 0 && q >= n3[a] - hi - 1);
    };
    for (size_t id = 0; id < nt; ++id) {
      const int bx = (int)(id % c->tgx), by = (int)((id / c->tgx) % c->tgy), bz = (int)(id / ((size_t)c->tgx * c->tgy));
      const int lo3[3] = {64 * bx, 4 * by, c->tkc * bz};
      const int hi3[3] = {std::min(64 * bx + 64, c->nx), std::min(4 * by + 4, c->ny), std::min(c->tkc * (bz + 1), c->nz)};
      bool hit = false;
      for (int a = 0; a < 3 && !hit; ++a)
        hit = band(a, lo3[a]) || band(a, hi3[a] - 1);
      pmlt[id] = hit;
    }
  }
  std::vector<int> all, nr, fr, pm;
  std::vector<unsigned char> far(nt, 0);
  c->cells_near = c->cells_far = 0;
  for (size_t id = 0; id < nt; ++id) {
    if (pmlt[id]) {
      pm.push_back((int)id);
      continue;
    }
    all.push_back((int)id);
    const int bx = (int)(id % c->tgx), by = (int)((id / c->tgx) % c->tgy), bz = (int)(id / ((size_t)c->tgx * c->tgy));
    const long long cells = (long long)std::min(64, c->nx - 64 * bx) * std::min(4, c->ny - 4 * by) *
                            std::min(c->tkc, c->nz - c->tkc * bz);
    if (near[id]) {
      nr.push_back((int)id);
      c->cells_near += cells;
    } else {
      fr.push_back((int)id);
      far[id] = 1;
      c->cells_far += cells;
    }
  }
  // pairs along y within each (x, z) tile column, greedily from the low row
  auto pairs = [&](const std::vector<int>& members, std::vector<int>& two, std::vector<int>& one) {
    std::vector<unsigned char> in(nt, 0);
    for (int id : members) in[id] = 1;
    for (int bz = 0; bz < c->tgz; ++bz)
      for (int bx = 0; bx < c->tgx; ++bx)
        for (int by = 0; by < c->tgy;) {
          const size_t id = (size_t)bx + (size_t)c->tgx * ((size_t)by + (size_t)c->tgy * bz);
          if (!in[id]) {
            ++by;
          } else if (by + 1 < c->tgy && in[id + c->tgx]) {
            two.push_back((int)id);
            by += 2;
          } else {
            one.push_back((int)id);
            ++by;
          }
        }
    std::sort(two.begin(), two.end());
    std::sort(one.begin(), one.end());
    two = xcd_order(two);
    one = xcd_order(one);
  };
  std::vector<int> all2, all1;
  pairs(all, all2, all1);
  all = xcd_order(all);
  nr = xcd_order(nr);
  fr = xcd_order(fr);
  pm = xcd_order(pm);
  {
    const std::vector<int>* src[2] = {&all2, &all1};
    int** dst[2] = {&c->d_tl_all2, &c->d_tl_all1};
    int* cnt[2] = {&c->n_all2, &c->n_all1};
    for (int q = 0; q < 2; ++q) {
      *dst[q] = (int*)dalloc(c, std::max<size_t>(src[q]->size(), 1) * sizeof(int));
      if (!*dst[q]) return fail(c, MM_ENOMEM, "tile-list allocation failed");
      if (!src[q]->empty())
        HIPCHECK(c, hipMemcpy(*dst[q], src[q]->data(), src[q]->size() * sizeof(int), hipMemcpyHostToDevice));
      *cnt[q] = (int)src[q]->size();
    }
  }
  c->n_pml = (int)pm.size();
  c->d_tl_pml = (int*)dalloc(c, std::max<size_t>(pm.size(), 1) * sizeof(int));
  if (!c->d_tl_pml) return fail(c, MM_ENOMEM, "tile-list allocation failed");
  if (!pm.empty()) HIPCHECK(c, hipMemcpy(c->d_tl_pml, pm.data(), pm.size() * sizeof(int), hipMemcpyHostToDevice));
  c->n_all = (int)all.size();
  c->n_near = (int)nr.size();
  c->n_far = (int)fr.size();
  c->d_tl_all = (int*)dalloc(c, std::max<size_t>(all.size(), 1) * sizeof(int));
  c->d_tl_near = (int*)dalloc(c, nr.size() * sizeof(int));
  c->d_tl_far = (int*)dalloc(c, fr.size() * sizeof(int));
  c->d_far = (unsigned char*)dalloc(c, nt);
  if (!c->d_tl_all || !c->d_tl_near || !c->d_tl_far || !c->d_far)
    return fail(c, MM_ENOMEM, "tile-list allocation failed");
  if (!all.empty()) HIPCHECK(c, hipMemcpy(c->d_tl_all, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice));
  if (!nr.empty()) HIPCHECK(c, hipMemcpy(c->d_tl_near, nr.data(), nr.size() * sizeof(int), hipMemcpyHostToDevice));
  if (!fr.empty()) HIPCHECK(c, hipMemcpy(c->d_tl_far, fr.data(), fr.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHECK(c, hipMemcpy(c->d_far, far.data(), nt, hipMemcpyHostToDevice));
  c->h_farv = far;
  return MM_OK;
}

// Chunks of the fused H-M sub-step: 30 x 6 columns x fL planes holding at
// least one evolving face, in XCD order, and for each chunk its slot table
// over the 32 x 8 x (fL + 2) cells of chunk and one-cell rim (per family:
// the face's list index and neighbour mask, or kNoFace).  fL is picked from
// 4..32 for the fewest chunk rounds over the CUs times pipeline steps.
mm_status build_fused(mm_ctx* c) {
  c->fused_ok = false;
  c->chain_fused = false;
  c->nchunks = 0;
  c->fL = 0;
  if (c->fuse_mode < 0 || c->scheme != 2 || c->nmag == 0 || c->has_pml) return MM_OK;
  if ((size_t)c->nmag + c->nwall >= (size_t(1) << 24)) return MM_OK;
  if (c->fuse_mode == 0 && c->nmag < (1 << 18)) return MM_OK;
  int dev = 0, ncu = 1;
  HIPCHECK(c, hipGetDevice(&dev));
  HIPCHECK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  using mmk::kFCols;
  using mmk::kFIX;
  using mmk::kFIY;
  using mmk::kFX;
  const int n3[3] = {c->nx, c->ny, c->nz};
  auto cell_of = [&](int t, int& i, int& j, int& k) {
    const int pi = c->h_idx[t];
    k = pi / (c->px * c->py);
    const int rr = pi - k * c->px * c->py;
    j = rr / c->px;
    i = rr - j * c->px;
  };
  auto chunks_for = [&](int L) {
    std::vector<long long> keys;
    keys.reserve(c->nmag / 16 + 16);
    const long long gx = (c->nx + kFIX - 1) / kFIX, gy = (c->ny + kFIY - 1) / kFIY;
    for (int t = 0; t < c->nmag; ++t) {
      int i, j, k;
      cell_of(t, i, j, k);
      keys.push_back((long long)(i / kFIX) + gx * ((long long)(j / kFIY) + gy * (long long)(k / L)));
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    return keys;
  };
  int bestL = 4;
  long long bestCost = -1;
  for (int L : {4, 8, 16, 32}) {
    const long long n = (long long)chunks_for(L).size();
    const long long cost = ((n + 2 * ncu - 1) / (2 * ncu)) * (L + 3);   // two chunks per CU
    if (bestCost < 0 || cost < bestCost) {
      bestCost = cost;
      bestL = L;
    }
  }
  const int L = bestL;
  const std::vector<long long> keys = chunks_for(L);
  std::vector<int> nat(keys.size());
  for (size_t q = 0; q < keys.size(); ++q) nat[q] = (int)q;
  const std::vector<int> ord = xcd_order(nat);
  const long long gx = (c->nx + kFIX - 1) / kFIX, gy = (c->ny + kFIY - 1) / kFIY;
  const int NC = (int)keys.size();
  std::vector<int> org(3 * (size_t)NC);
  for (int b = 0; b < NC; ++b) {
    const long long key = keys[ord[b]];
    org[3 * b] = (int)(key % gx) * kFIX;
    org[3 * b + 1] = (int)((key / gx) % gy) * kFIY;
    org[3 * b + 2] = (int)(key / (gx * gy)) * L;
  }
  // face lookup: (family, padded index) -> list index of the evolving face
  const bool dense = c->nelem <= (size_t(64) << 20);
  std::vector<int> dmap;
  std::unordered_map<long long, int> hmap;
  if (dense) {
    dmap.assign(3 * c->nelem, -1);
    for (int t = 0; t < c->nmag; ++t) dmap[(size_t)c->h_fam[t] * c->nelem + c->h_idx[t]] = t;
  } else {
    hmap.reserve((size_t)c->nmag * 2);
    for (int t = 0; t < c->nmag; ++t) hmap[(long long)c->h_fam[t] * (long long)c->nelem + c->h_idx[t]] = t;
  }
  auto lookup = [&](int f, size_t pi) -> int {
    if (dense) return dmap[(size_t)f * c->nelem + pi];
    auto it = hmap.find((long long)f * (long long)c->nelem + (long long)pi);
    return it == hmap.end() ? -1 : it->second;
  };
  const int EP = L + 2;
  const size_t per_chunk = (size_t)EP * 3 * kFCols;
  std::vector<unsigned> slots(per_chunk * NC, mmk::kNoFace);
  for (int b = 0; b < NC; ++b) {
    unsigned* sl = slots.data() + per_chunk * b;
    for (int e = 0; e < EP; ++e)
      for (int col = 0; col < kFCols; ++col) {
        const int u[3] = {org[3 * b] - 1 + col % kFX, org[3 * b + 1] - 1 + col / kFX, org[3 * b + 2] - 1 + e};
        int w[3];
        bool ok = true;
        for (int a = 0; a < 3 && ok; ++a) {
          if (c->per >> a & 1) w[a] = ((u[a] % n3[a]) + n3[a]) % n3[a];
          else if (u[a] < 0 || u[a] >= n3[a]) ok = false;
          else w[a] = u[a];
        }
        if (!ok) continue;
        const size_t pi = pidx(c, w[0], w[1], w[2]);
        for (int f = 0; f < 3; ++f) {
          const int t = lookup(f, pi);
          if (t >= 0) sl[((size_t)e * 3 + f) * kFCols + col] = ((unsigned)t << 8) | c->h_nbm[t];
        }
      }
  }
  c->d_forg = (int*)dalloc(c, org.size() * sizeof(int));
  c->d_fslots = (unsigned*)dalloc(c, slots.size() * sizeof(unsigned));
  c->d_fpart = (unsigned long long*)dalloc(c, 2 * 4 * (size_t)NC * sizeof(unsigned long long));
  c->d_kpred = (int*)dalloc(c, sizeof(int));
  const size_t ntot = (size_t)c->nmag + c->nwall;
  for (int a = 0; a < 3; ++a) {
    c->d_Mb[a] = (double*)dalloc(c, ntot * sizeof(double));
    if (!c->d_Mb[a]) return fail(c, MM_ENOMEM, "allocation of the second M buffer failed");
    HIPCHECK(c, hipMemcpy(c->d_Mb[a], c->d_M[a], ntot * sizeof(double), hipMemcpyDeviceToDevice));
  }
  if (!c->d_forg || !c->d_fslots || !c->d_fpart || !c->d_kpred)
    return fail(c, MM_ENOMEM, "allocation of the fused sub-step tables failed");
  HIPCHECK(c, hipMemcpy(c->d_forg, org.data(), org.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHECK(c, hipMemcpy(c->d_fslots, slots.data(), slots.size() * sizeof(unsigned), hipMemcpyHostToDevice));
  HIPCHECK(c, hipMemset(c->d_fpart, 0, 2 * 4 * (size_t)NC * sizeof(unsigned long long)));
  const int one = 1;
  HIPCHECK(c, hipMemcpy(c->d_kpred, &one, sizeof(int), hipMemcpyHostToDevice));
  c->ctl_kpred = c->d_kpred;
  c->ctl_fpart = c->d_fpart;
  c->nchunks = NC;
  c->fL = L;
  c->fused_ok = true;
  return MM_OK;
}

mm_status build(mm_ctx* c, const mm_materials* mat, const mm_source* src) {
  const size_t ncells = (size_t)c->nx * c->ny * c->nz;
  const bool fp32 = c->prec == MM_FP32;
  // fields
  for (int a = 0; a < 3; ++a) {
    c->E[a] = dalloc(c, c->nelem * c->esz);
    c->H[a] = dalloc(c, c->nelem * c->esz);
    if (!c->E[a] || !c->H[a]) return fail(c, MM_ENOMEM, "device allocation of the fields failed");
    HIPCHECK(c, hipMemsetAsync(c->E[a], 0, c->nelem * c->esz, c->stream));
    HIPCHECK(c, hipMemsetAsync(c->H[a], 0, c->nelem * c->esz, c->stream));
  }
  // cell maps: eps always; sigma only if some cell conducts; mu only if some mu_r != 1
  bool any_sig = false, any_mu = false;
  if (mat->sigma)
    for (size_t q = 0; q < ncells && !any_sig; ++q) any_sig = mat->sigma[q] != 0.0;
  if (mat->mu_r)
    for (size_t q = 0; q < ncells && !any_mu; ++q) any_mu = mat->mu_r[q] != 1.0;
  mm_status s;
  s = fp32 ? upload_cellmap<float>(c, mat->eps_r, 1.0, &c->eps) : upload_cellmap<double>(c, mat->eps_r, 1.0, &c->eps);
  if (s) return s;
  if (any_sig) {
    s = fp32 ? upload_cellmap<float>(c, mat->sigma, 0.0, &c->sig) : upload_cellmap<double>(c, mat->sigma, 0.0, &c->sig);
    if (s) return s;
  }
  if (any_mu) {
    s = fp32 ? upload_cellmap<float>(c, mat->mu_r, 1.0, &c->mu) : upload_cellmap<double>(c, mat->mu_r, 1.0, &c->mu);
    if (s) return s;
  }
  s = fp32 ? build_material_ids<float>(c, mat) : build_material_ids<double>(c, mat);
  if (s) return s;

  // magnetic faces: Ms_f = mean of the 2 cells (a PEC wall face uses its one
  // cell); alpha_f, gamma_f over the magnetic cells only; M0_f = mean of
  // Ms*m0_dir renormalised to Ms_f (Sec. 3.1).
  std::vector<int> ev_idx[3], wl_idx[3];
  std::vector<double> ev_v[3][7], wl_v[3][7];  // Ms, kap, aoms, M0x, M0y, M0z, unused
  std::vector<FaceCells> ev_fc[3], wl_fc[3];
  c->cell_mag.assign(ncells, false);
  if (mat->Ms)
    for (size_t q = 0; q < ncells; ++q) c->cell_mag[q] = mat->Ms[q] > 0;
  for (int f = 0; f < 3; ++f) {
    int ext[3];
    field_extent(c, 3 + f, ext);
    const bool pf = c->per >> f & 1;
    const int nf = ncell(c, f);
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) {
          int p[3] = {i, j, k};
          int qa[3] = {i, j, k}, qb[3] = {i, j, k};
          bool wall = false;
          // the two cells sharing the face: index-1 and index along f
          qa[f] = p[f] - 1;
          qb[f] = p[f];
          if (pf) {
            if (qa[f] < 0) qa[f] = nf - 1;
          } else {
            if (p[f] == 0) { qa[f] = 0; wall = true; }
            if (p[f] == nf) { qb[f] = nf - 1; wall = true; }
          }
          const double msa = cell(mat->Ms, 0.0, c, qa[0], qa[1], qa[2]);
          const double msb = cell(mat->Ms, 0.0, c, qb[0], qb[1], qb[2]);
          double Msf;
          if (wall) {
            const double v = (p[f] == 0) ? msb : msa;
            Msf = 0.5 * (2.0 * v);
          } else {
            Msf = 0.5 * (msa + msb);
          }
          if (!(Msf > 0)) continue;
          const double ma = msa > 0 ? 1.0 : 0.0, mb = msb > 0 ? 1.0 : 0.0;
          const double aa = cell(mat->alpha, 0.0, c, qa[0], qa[1], qa[2]);
          const double ab = cell(mat->alpha, 0.0, c, qb[0], qb[1], qb[2]);
          const double ga = cell(mat->gamma, -1.759e11, c, qa[0], qa[1], qa[2]);
          const double gb = cell(mat->gamma, -1.759e11, c, qb[0], qb[1], qb[2]);
          double af, gf, M0[3];
          const size_t ncell_all = ncells;
          auto mdir = [&](int comp, const int q[3]) {
            if (!mat->m0_dir) return comp == 2 ? 1.0 : 0.0;
            return mat->m0_dir[(size_t)comp * ncell_all + (size_t)q[0] + (size_t)c->nx * ((size_t)q[1] + (size_t)c->ny * (size_t)q[2])];
          };
          if (wall) {
            const int* q = (p[f] == 0) ? qb : qa;
            const double m = (p[f] == 0) ? mb : ma;
            const double al = (p[f] == 0) ? ab : aa;
            const double ga1 = (p[f] == 0) ? gb : ga;
            const double ms = (p[f] == 0) ? msb : msa;
            af = (2.0 * al * m) / (2.0 * m);
            gf = (2.0 * ga1 * m) / (2.0 * m);
            for (int cc = 0; cc < 3; ++cc) M0[cc] = 0.5 * (2.0 * (ms * mdir(cc, q)));
          } else {
            const double cnt = ma + mb;
            af = (aa * ma + ab * mb) / cnt;
            gf = (ga * ma + gb * mb) / cnt;
            for (int cc = 0; cc < 3; ++cc) M0[cc] = 0.5 * (msa * mdir(cc, qa) + msb * mdir(cc, qb));
          }
          const double nrm = std::sqrt((M0[0] * M0[0] + M0[1] * M0[1]) + M0[2] * M0[2]);
          if (!(nrm > 0)) return fail(c, MM_EINVAL, "initial magnetisation averages to zero on a magnetic face");
          const double sc = Msf / nrm;
          // per-face constants of the sub-step: kappa = mu0 gamma dt / 4 and
          // alpha / Ms (eq:llg_tra5/6), or for the first-order scheme
          // mu0 gamma_L and alpha mu0 gamma_L / Ms (eq:LLG_scalar)
          double k1 = mmk::kMu0 * gf * c->dt / 4.0, k2 = af / Msf;
          if (c->scheme == 1) {
            const double gL = gf / (1.0 + af * af);
            k1 = mmk::kMu0 * gL;
            k2 = af * mmk::kMu0 * gL / Msf;
          }
          const double vals[7] = {Msf, k1, k2, M0[0] * sc, M0[1] * sc, M0[2] * sc, 0.0};
          const int pi = (int)pidx(c, i, j, k);
          FaceCells fcl;
          auto lin = [&](const int q[3]) {
            return (long long)q[0] + (long long)c->nx * ((long long)q[1] + (long long)c->ny * q[2]);
          };
          if (wall) {
            const int* q = (p[f] == 0) ? qb : qa;
            fcl.a = lin(q);
            fcl.b = -1;
            for (int cc = 0; cc < 3; ++cc) {
              fcl.ma[cc] = mdir(cc, q);
              fcl.mb[cc] = 0.0;
            }
          } else {
            fcl.a = lin(qa);
            fcl.b = lin(qb);
            for (int cc = 0; cc < 3; ++cc) {
              fcl.ma[cc] = mdir(cc, qa);
              fcl.mb[cc] = mdir(cc, qb);
            }
          }
          for (int cc = 0; cc < 3; ++cc) fcl.v[cc] = M0[cc];
          if (wall) {
            wl_idx[f].push_back(pi);
            for (int v = 0; v < 7; ++v) wl_v[f][v].push_back(vals[v]);
            wl_fc[f].push_back(fcl);
          } else {
            ev_idx[f].push_back(pi);
            for (int v = 0; v < 7; ++v) ev_v[f][v].push_back(vals[v]);
            ev_fc[f].push_back(fcl);
          }
        }
  }
  c->off1 = (int)ev_idx[0].size();
  c->off2 = c->off1 + (int)ev_idx[1].size();
  c->nmag = c->off2 + (int)ev_idx[2].size();
  c->nwall = (int)(wl_idx[0].size() + wl_idx[1].size() + wl_idx[2].size());
  const size_t ntot = (size_t)c->nmag + c->nwall;
  std::vector<double> hv[7];
  c->h_idx.clear();
  c->h_fam.clear();
  c->fcells.clear();
  for (int f = 0; f < 3; ++f) c->fcells.insert(c->fcells.end(), ev_fc[f].begin(), ev_fc[f].end());
  for (int f = 0; f < 3; ++f) c->fcells.insert(c->fcells.end(), wl_fc[f].begin(), wl_fc[f].end());
  for (int f = 0; f < 3; ++f) {
    c->h_idx.insert(c->h_idx.end(), ev_idx[f].begin(), ev_idx[f].end());
    c->h_fam.insert(c->h_fam.end(), ev_idx[f].size(), f);
    for (int v = 0; v < 7; ++v) hv[v].insert(hv[v].end(), ev_v[f][v].begin(), ev_v[f][v].end());
  }
  for (int f = 0; f < 3; ++f) {
    c->h_idx.insert(c->h_idx.end(), wl_idx[f].begin(), wl_idx[f].end());
    c->h_fam.insert(c->h_fam.end(), wl_idx[f].size(), f);
    for (int v = 0; v < 7; ++v) hv[v].insert(hv[v].end(), wl_v[f][v].begin(), wl_v[f][v].end());
  }
  if (ntot > 0) {
    c->d_idx = (int*)dalloc(c, ntot * sizeof(int));
    c->d_Ms = (double*)dalloc(c, ntot * sizeof(double));
    c->d_kap = (double*)dalloc(c, ntot * sizeof(double));
    c->d_aoms = (double*)dalloc(c, ntot * sizeof(double));
    for (int a = 0; a < 3; ++a) {
      c->d_M[a] = (double*)dalloc(c, ntot * sizeof(double));
      c->d_b[a] = (double*)dalloc(c, ntot * sizeof(double));
      c->d_d[a] = (double*)dalloc(c, ntot * sizeof(double));
      if (!c->d_M[a] || !c->d_b[a] || !c->d_d[a]) return fail(c, MM_ENOMEM, "magnetic-face allocation failed");
    }
    c->d_q = (double*)dalloc(c, ntot * sizeof(double));
    c->d_nbm = (unsigned char*)dalloc(c, ntot);
    if (!c->d_idx || !c->d_Ms || !c->d_kap || !c->d_aoms || !c->d_q || !c->d_nbm)
      return fail(c, MM_ENOMEM, "magnetic-face allocation failed");
    for (int a = 0; a < 3; ++a) {
      c->A[a] = dalloc(c, c->nelem * c->esz);
      c->B[a] = dalloc(c, c->nelem * c->esz);
      if (!c->A[a] || !c->B[a]) return fail(c, MM_ENOMEM, "allocation of the shadow H failed");
      HIPCHECK(c, hipMemsetAsync(c->A[a], 0, c->nelem * c->esz, c->stream));
      HIPCHECK(c, hipMemsetAsync(c->B[a], 0, c->nelem * c->esz, c->stream));
    }
    // neighbour masks: bit q set when transverse neighbour q (numbered as in
    // mmk::h_eff) is an evolving magnetic face
    {
      std::vector<std::vector<bool>> ev(3, std::vector<bool>(c->nelem, false));
      for (size_t t = 0; t < (size_t)c->nmag; ++t) ev[c->h_fam[t]][c->h_idx[t]] = true;
      std::vector<unsigned char> nbm(ntot, 0);
      auto dn = [&](int i, int n, bool p) { return (p && i == 0) ? n - 1 : i - 1; };
      auto up = [&](int i, int n, bool p) { return (p && i == n - 1) ? 0 : i + 1; };
      const bool pxp = c->per & 1, pyp = c->per & 2, pzp = c->per & 4;
      for (size_t t = 0; t < (size_t)c->nmag; ++t) {
        const int pi = c->h_idx[t], f = c->h_fam[t];
        const int k = pi / (c->px * c->py), rr = pi - k * c->px * c->py, j = rr / c->px, i = rr - j * c->px;
        int comp[8], ii[8], jj[8], kk[8];
        auto set = [&](int q, int cp, int a, int b2, int d2) { comp[q] = cp; ii[q] = a; jj[q] = b2; kk[q] = d2; };
        if (f == 0) {
          const int im = dn(i, c->nx, pxp), jp = up(j, c->ny, pyp), kp = up(k, c->nz, pzp);
          set(0, 1, im, j, k); set(1, 1, i, j, k); set(2, 1, im, jp, k); set(3, 1, i, jp, k);
          set(4, 2, im, j, k); set(5, 2, i, j, k); set(6, 2, im, j, kp); set(7, 2, i, j, kp);
        } else if (f == 1) {
          const int jm = dn(j, c->ny, pyp), ip = up(i, c->nx, pxp), kp = up(k, c->nz, pzp);
          set(0, 0, i, jm, k); set(1, 0, i, j, k); set(2, 0, ip, jm, k); set(3, 0, ip, j, k);
          set(4, 2, i, jm, k); set(5, 2, i, j, k); set(6, 2, i, jm, kp); set(7, 2, i, j, kp);
        } else {
          const int km = dn(k, c->nz, pzp), ip = up(i, c->nx, pxp), jp = up(j, c->ny, pyp);
          set(0, 0, i, j, km); set(1, 0, i, j, k); set(2, 0, ip, j, km); set(3, 0, ip, j, k);
          set(4, 1, i, j, km); set(5, 1, i, j, k); set(6, 1, i, jp, km); set(7, 1, i, jp, k);
        }
        unsigned char mk = 0;
        for (int q = 0; q < 8; ++q)
          if (ev[comp[q]][pidx(c, ii[q], jj[q], kk[q])]) mk |= (unsigned char)(1u << q);
        nbm[t] = mk;
      }
      HIPCHECK(c, hipMemcpy(c->d_nbm, nbm.data(), ntot, hipMemcpyHostToDevice));
      c->h_nbm = nbm;
    }
    HIPCHECK(c, hipMemcpy(c->d_idx, c->h_idx.data(), ntot * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->d_Ms, hv[0].data(), ntot * sizeof(double), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->d_kap, hv[1].data(), ntot * sizeof(double), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->d_aoms, hv[2].data(), ntot * sizeof(double), hipMemcpyHostToDevice));
    for (int a = 0; a < 3; ++a)
      HIPCHECK(c, hipMemcpy(c->d_M[a], hv[3 + a].data(), ntot * sizeof(double), hipMemcpyHostToDevice));
    // face materials: the distinct (Ms, kap, aoms) triples of the evolving
    // faces (bit-exact), a byte id per face when there are at most 256
    c->d_fid = nullptr;
    c->d_ftab = nullptr;
    c->nfmat = 0;
    if (c->nmag > 0) {
      std::map<std::array<uint64_t, 3>, int> ids;
      std::vector<unsigned char> fid(c->nmag);
      std::vector<double> tab;
      bool fits = true;
      for (size_t t = 0; t < (size_t)c->nmag && fits; ++t) {
        std::array<uint64_t, 3> key;
        for (int v = 0; v < 3; ++v) std::memcpy(&key[v], &hv[v][t], sizeof(double));
        auto it = ids.find(key);
        if (it == ids.end()) {
          if (ids.size() == 256) {
            fits = false;
            break;
          }
          it = ids.emplace(key, (int)ids.size()).first;
          for (int v = 0; v < 3; ++v) tab.push_back(hv[v][t]);
        }
        fid[t] = (unsigned char)it->second;
      }
      if (fits) {
        c->nfmat = (int)ids.size();
        c->d_fid = (unsigned char*)dalloc(c, c->nmag);
        c->d_ftab = (double*)dalloc(c, tab.size() * sizeof(double));
        if (!c->d_fid || !c->d_ftab) return fail(c, MM_ENOMEM, "face-material allocation failed");
        HIPCHECK(c, hipMemcpy(c->d_fid, fid.data(), c->nmag, hipMemcpyHostToDevice));
        HIPCHECK(c, hipMemcpy(c->d_ftab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
      }
    }
  }
  c->nres = std::max(c->max_iter, c->fixed_iter) + 2;
  c->step_blocks = c->fin_blocks = 1;
  if (c->nmag > 0) {
    int dev = 0, ncu = 0;
    HIPCHECK(c, hipGetDevice(&dev));
    HIPCHECK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int want = (c->nmag + MM_MAG_THREADS - 1) / MM_MAG_THREADS;
    c->step_blocks = std::max(1, std::min(want, MM_MAG_BLOCKS_PER_CU * ncu));
    // hm_finish: co-resident (at most one block per CU) and no more blocks
    // than residual slots, so that every slot has an owner
    c->fin_blocks = std::max(1, std::min(c->step_blocks, ncu));
  }
  c->d_res = (unsigned long long*)dalloc(c, 2 * sizeof(unsigned long long));
  c->d_part = (unsigned long long*)dalloc(c, 2 * (size_t)c->nres * c->step_blocks * sizeof(unsigned long long));
  c->d_err = (int*)dalloc(c, sizeof(int));
  c->d_bar = (unsigned int*)dalloc(c, 2 * sizeof(unsigned int));
  if (!c->d_res || !c->d_part || !c->d_err || !c->d_bar) return fail(c, MM_ENOMEM, "allocation failed");
  HIPCHECK(c, hipMemset(c->d_res, 0, 2 * sizeof(unsigned long long)));
  HIPCHECK(c, hipMemset(c->d_part, 0, 2 * (size_t)c->nres * c->step_blocks * sizeof(unsigned long long)));
  HIPCHECK(c, hipMemset(c->d_err, 0, sizeof(int)));
  HIPCHECK(c, hipMemset(c->d_bar, 0, 2 * sizeof(unsigned int)));
  c->ctl_res = c->d_res;
  c->ctl_part = c->d_part;
  c->ctl_bar = c->d_bar;
  {
    mm_status fs = build_fused(c);
    if (fs) return fs;
  }
  HIPCHECK(c, hipHostMalloc((void**)&c->h_ring, 64 * sizeof(int), hipHostMallocMapped));
  std::memset(c->h_ring, 0, 64 * sizeof(int));
  HIPCHECK(c, hipHostGetDevicePointer((void**)&c->d_ring, c->h_ring, 0));

  {
    mm_status ts = upload_pml(c);
    if (ts) return ts;
    ts = build_tiles(c);
    if (ts) return ts;
  }

  // soft source: J0 p over the bounding box of its nonzero interior edges
  c->nsrc = 0;
  if (src && src->profile) {
    const int cp = src->comp;
    int ext[3];
    field_extent(c, cp, ext);
    int lo[3] = {ext[0], ext[1], ext[2]}, hi[3] = {0, 0, 0};
    auto prof_at = [&](int i, int j, int k) {
      return src->profile[(size_t)i + (size_t)ext[0] * ((size_t)j + (size_t)ext[1] * k)];
    };
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) {
          if (prof_at(i, j, k) == 0.0 || !entry_interior(c, cp, i, j, k)) continue;
          c->nsrc++;
          const int p[3] = {i, j, k};
          for (int a2 = 0; a2 < 3; ++a2) {
            lo[a2] = std::min(lo[a2], p[a2]);
            hi[a2] = std::max(hi[a2], p[a2] + 1);
          }
        }
    if (c->nsrc) {
      const size_t bx = hi[0] - lo[0], by = hi[1] - lo[1], bz = hi[2] - lo[2];
      std::vector<double> box(bx * by * bz, 0.0);
      for (size_t k = 0; k < bz; ++k)
        for (size_t j = 0; j < by; ++j)
          for (size_t i = 0; i < bx; ++i) {
            const int gi = lo[0] + (int)i, gj = lo[1] + (int)j, gk = lo[2] + (int)k;
            if (entry_interior(c, cp, gi, gj, gk)) box[i + bx * (j + by * k)] = prof_at(gi, gj, gk);
          }
      c->d_src_prof = (double*)dalloc(c, box.size() * sizeof(double));
      if (!c->d_src_prof) return fail(c, MM_ENOMEM, "source allocation failed");
      HIPCHECK(c, hipMemcpy(c->d_src_prof, box.data(), box.size() * sizeof(double), hipMemcpyHostToDevice));
      for (int a2 = 0; a2 < 3; ++a2) {
        c->src_lo[a2] = lo[a2];
        c->src_hi[a2] = hi[a2];
      }
    }
    c->src_comp = cp;
    c->f0 = src->f0;
    c->Tp = src->Tp;
    c->t0 = src->t0;
  }
  return MM_OK;
}

#include "adjoint_host.h"

void release(mm_ctx* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (auto& pr : c->ev_pool) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  c->ev_pool.clear();
  if (c->h_ring) {
    (void)hipHostFree(c->h_ring);
    c->h_ring = nullptr;
  }
  while (!c->allocs.empty()) dfree(c, c->allocs.back().first);
  delete c->adjw;
  c->adjw = nullptr;
}

}  // namespace

extern "C" {

mm_status mm_init(mm_ctx** out, const mm_grid* g, double dt, const mm_materials* mat, const mm_bias* bias,
                  const mm_source* src, const mm_options* opt) {
  if (!out) return MM_EINVAL;
  *out = nullptr;
  if (!g || !mat || !opt) return MM_EINVAL;
  mm_ctx* c = new mm_ctx();
  auto bad = [&](const char* msg) {
    delete c;
    (void)msg;
    return MM_EINVAL;
  };
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return bad("grid");
  for (int a = 0; a < 3; ++a)
    if (g->bc[a] != MM_BC_PEC && g->bc[a] != MM_BC_PERIODIC) return bad("bc");
  if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) || !std::isfinite(g->dx + g->dy + g->dz)) return bad("spacing");
  const double dtmax = 1.0 / (kC0 * std::sqrt(1.0 / (g->dx * g->dx) + 1.0 / (g->dy * g->dy) + 1.0 / (g->dz * g->dz)));
  if (!(dt > 0) || !(dt <= dtmax * (1.0 + 1e-12))) return bad("dt");
  if (!(opt->tol > 0) || opt->max_iter < 1 || opt->fixed_iter < 0 || opt->fixed_iter > 1000000 ||
      opt->max_iter > 1000000)
    return bad("iteration options");
  if (opt->prec != MM_FP64 && opt->prec != MM_FP32) return bad("precision");
  if (opt->scheme != 0 && opt->scheme != 1 && opt->scheme != 2) return bad("scheme");
  if (opt->fused < -1 || opt->fused > 1) return bad("fused");
  if (opt->pml) {
    const int n3[3] = {g->nx, g->ny, g->nz};
    bool any = false;
    for (int a = 0; a < 3; ++a) {
      const int lo = opt->pml->cells[2 * a], hi = opt->pml->cells[2 * a + 1];
      if (lo < 0 || hi < 0 || lo + hi >= n3[a]) return bad("PML thickness");
      if ((lo || hi) && g->bc[a] == MM_BC_PERIODIC) return bad("PML on a periodic axis");
      any = any || lo || hi;
    }
    if (any && (!(opt->pml->R0 > 0 && opt->pml->R0 < 1) || !(opt->pml->order >= 1))) return bad("PML grading");
  }
  const size_t ncells = (size_t)g->nx * g->ny * g->nz;
  if (!finite_nonneg(mat->eps_r, ncells, true) || !finite_nonneg(mat->mu_r, ncells, true) ||
      !finite_nonneg(mat->sigma, ncells, false) || !finite_nonneg(mat->Ms, ncells, false) ||
      !finite_nonneg(mat->alpha, ncells, false))
    return bad("material map");
  if (mat->gamma)
    for (size_t q = 0; q < ncells; ++q)
      if (!std::isfinite(mat->gamma[q])) return bad("gamma");
  if (mat->m0_dir)
    for (size_t q = 0; q < 3 * ncells; ++q)
      if (!std::isfinite(mat->m0_dir[q])) return bad("m0_dir");
  if (src && src->profile) {
    if (src->comp < 0 || src->comp > 2 || !(src->Tp > 0) || !std::isfinite(src->f0) || !std::isfinite(src->t0))
      return bad("source");
  }
  c->nx = g->nx;
  c->ny = g->ny;
  c->nz = g->nz;
  c->per = (g->bc[0] == MM_BC_PERIODIC ? 1 : 0) | (g->bc[1] == MM_BC_PERIODIC ? 2 : 0) |
           (g->bc[2] == MM_BC_PERIODIC ? 4 : 0);
  c->dx = g->dx;
  c->dy = g->dy;
  c->dz = g->dz;
  c->dt = dt;
  c->px = ((c->nx + 1) + 31) / 32 * 32;
  c->py = c->ny + 1;
  c->pz = c->nz + 1;
  const double ne = (double)c->px * c->py * c->pz;
  if (ne >= 2147483647.0) return bad("grid too large for 32-bit indexing");
  c->nelem = (size_t)c->px * c->py * c->pz;
  c->prec = opt->prec;
  c->esz = opt->prec == MM_FP32 ? 4 : 8;
  c->tol = opt->tol;
  c->max_iter = opt->max_iter;
  c->fixed_iter = opt->fixed_iter;
  c->scheme = opt->scheme == 1 ? 1 : 2;
  c->fuse_mode = opt->fused;
  if (c->scheme == 1) c->fixed_iter = 1;   // one explicit update per sub-step
  for (int a = 0; a < 3; ++a) c->H0[a] = bias ? bias->H0[a] : 0.0;
  c->stream = (hipStream_t)opt->hip_stream;
  c->ualloc = opt->dev_alloc;
  c->ufree = opt->dev_free;
  c->actx = opt->alloc_ctx;
  resolve_scratch(c);
  mm_status s = setup_pml(c, opt->pml);
  if (s == MM_OK) s = build(c, mat, src);
  if (s == MM_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = fail(c, MM_EDEVICE, "init: %s", hipGetErrorString(e));
  }
  if (s != MM_OK) {
    std::fprintf(stderr, "mm_init: %s\n", c->err.c_str());
    release(c);
    delete c;
    return s;
  }
  *out = c;
  return MM_OK;
}

mm_status mm_step(mm_ctx* c, int64_t n) {
  if (!c) return MM_EINVAL;
  if (n < 0) return fail(c, MM_EINVAL, "negative step count");
  if (n == 0) return MM_OK;
  mm_status s = freeze_probes(c);
  if (s) return s;
  s = grow_buffers(c, (size_t)(c->step + n));
  if (s) return s;
  return c->prec == MM_FP32 ? run_steps<float>(c, n) : run_steps<double>(c, n);
}

mm_status mm_step_noalloc(mm_ctx* c, int64_t n) {
  if (!c) return MM_EINVAL;
  if (n < 0) return fail(c, MM_EINVAL, "negative step count");
  if (n == 0) return MM_OK;
  if (!c->scratch)
    return fail(c, MM_EDEVICE, "mm_step_noalloc: the fixed device storage was not resolved at init (%s)",
                c->scratch_err.c_str());
  if (!c->probes.empty() && !c->probes_frozen)
    return fail(c, MM_ESTATE, "mm_step_noalloc: probes added since the last mm_step have no storage yet "
                              "(mm_step creates it)");
  if (c->ckpt_every > 0)
    return fail(c, MM_ESTATE, "mm_step_noalloc: adjoint checkpoints are enabled; they need mm_step");
  const size_t need = (size_t)c->step + (size_t)n;
  const size_t cap_steps = std::min(c->iters_cap / 2, c->probes.empty() ? SIZE_MAX : c->series_cap);
  if (need > cap_steps)
    return fail(c, MM_EINVAL,
                "mm_step_noalloc: %lld steps would end at step %zu, beyond the iteration-log and probe "
                "storage made by earlier mm_step calls (%zu steps)",
                (long long)n, need, cap_steps);
  const size_t bytes = ctl_bytes(c);
  if (bytes > kScratchBytes)
    return fail(c, MM_EINVAL,
                "mm_step_noalloc: the sub-step control needs %zu bytes (max_iter %d, %d blocks), above the "
                "fixed %zu bytes",
                bytes, c->max_iter, c->step_blocks, kScratchBytes);
  unsigned char* base = (unsigned char*)c->scratch;
  // the final-count words and the barrier state start at zero; the
  // partials are written before they are read
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, c->stream, (unsigned int*)base,
                     (int)(kScratchHeader / sizeof(unsigned int)));
  HIPCHECK(c, hipGetLastError());
  unsigned long long* res = c->ctl_res;
  unsigned long long* part = c->ctl_part;
  unsigned int* bar = c->ctl_bar;
  int* kpred = c->ctl_kpred;
  unsigned long long* fpart = c->ctl_fpart;
  c->ctl_res = (unsigned long long*)base;
  c->ctl_bar = (unsigned int*)(base + 64);
  c->ctl_part = (unsigned long long*)(base + kScratchHeader);
  if (c->fused_ok) {
    // the fused form's count prediction carries over from the context
    c->ctl_kpred = (int*)(base + 128);
    c->ctl_fpart = c->ctl_part + 2 * (size_t)c->nres * c->step_blocks;
    hipLaunchKernelGGL(copy_word, dim3(1), dim3(64), 0, c->stream, c->ctl_kpred, kpred);
  }
  const mm_status s = c->prec == MM_FP32 ? run_steps<float>(c, n) : run_steps<double>(c, n);
  if (c->fused_ok) hipLaunchKernelGGL(copy_word, dim3(1), dim3(64), 0, c->stream, kpred, c->ctl_kpred);
  c->ctl_res = res;
  c->ctl_part = part;
  c->ctl_bar = bar;
  c->ctl_kpred = kpred;
  c->ctl_fpart = fpart;
  return s;
}

namespace {

// Register a hard source on component `field` (0-5) from a host profile on
// its staggered extent; see mm_add_hard_source for the conditions.
mm_status add_hard(mm_ctx* c, int field, const double* profile, double f0, double Tp, double t0) {
  if (c->step > 0 || c->substep > 0) return fail(c, MM_ESTATE, "hard sources must be added before the first step");
  if (c->ckpt_every > 0) return fail(c, MM_EINVAL, "the adjoint does not cover hard sources");
  if (field < 0 || field > 5 || !profile) return fail(c, MM_EINVAL, "bad hard source (field %d)", field);
  if (!(Tp > 0) || !std::isfinite(f0) || !std::isfinite(t0)) return fail(c, MM_EINVAL, "bad hard source pulse");
  if ((int)c->hard.size() >= MM_MAX_HARD) return fail(c, MM_EINVAL, "at most %d hard sources", MM_MAX_HARD);
  int ext[3];
  field_extent(c, field, ext);
  auto prof_at = [&](int i, int j, int k) {
    return profile[(size_t)i + (size_t)ext[0] * ((size_t)j + (size_t)ext[1] * k)];
  };
  int lo[3] = {ext[0], ext[1], ext[2]}, hi[3] = {0, 0, 0};
  bool any = false;
  for (int k = 0; k < ext[2]; ++k)
    for (int j = 0; j < ext[1]; ++j)
      for (int i = 0; i < ext[0]; ++i) {
        const double v = prof_at(i, j, k);
        if (!std::isfinite(v)) return fail(c, MM_EINVAL, "non-finite hard source profile");
        if (v == 0.0 || !entry_interior(c, field, i, j, k)) continue;
        any = true;
        const int p[3] = {i, j, k};
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], p[a]);
          hi[a] = std::max(hi[a], p[a] + 1);
        }
      }
  if (!any) return fail(c, MM_EINVAL, "a hard source needs a nonzero interior profile entry");
  if (field >= 3) {
    const int f = field - 3;
    const int t0f = f == 0 ? 0 : (f == 1 ? c->off1 : c->off2);
    const int t1f = f == 0 ? c->off1 : (f == 1 ? c->off2 : c->nmag);
    for (int t = t0f; t < t1f; ++t) {
      const size_t pi = (size_t)c->h_idx[t];
      const int k = (int)(pi / ((size_t)c->px * c->py));
      const size_t rr = pi - (size_t)k * c->px * c->py;
      const int j = (int)(rr / c->px), i = (int)(rr % c->px);
      if (i >= lo[0] && i < hi[0] && j >= lo[1] && j < hi[1] && k >= lo[2] && k < hi[2])
        return fail(c, MM_EINVAL, "a hard H source may not hold evolving magnetic faces");
    }
  }
  if (c->has_pml) {
    const int n3[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
      const int lt = c->pml_cells[2 * a], ht = c->pml_cells[2 * a + 1];
      // positions in cells: cell centres where the component is cell-centred
      const bool cell_axis = field < 3 ? a == field : a != field - 3;
      for (int q = lo[a]; q < hi[a]; ++q) {
        const double pos = q + (cell_axis ? 0.5 : 0.0);
        if ((lt > 0 && pos < lt) || (ht > 0 && pos > n3[a] - ht))
          return fail(c, MM_EINVAL, "a hard source may not reach into an open-boundary layer");
      }
    }
  }
  HardSrc hs;
  hs.field = field;
  for (int a = 0; a < 3; ++a) {
    hs.lo[a] = lo[a];
    hs.n[a] = hi[a] - lo[a];
  }
  hs.f0 = f0;
  hs.Tp = Tp;
  hs.t0 = t0;
  const size_t bx = hs.n[0], by = hs.n[1], bz = hs.n[2];
  std::vector<double> box(bx * by * bz, 0.0);
  for (size_t k = 0; k < bz; ++k)
    for (size_t j = 0; j < by; ++j)
      for (size_t i = 0; i < bx; ++i) {
        const int gi = lo[0] + (int)i, gj = lo[1] + (int)j, gk = lo[2] + (int)k;
        if (entry_interior(c, field, gi, gj, gk)) box[i + bx * (j + by * k)] = prof_at(gi, gj, gk);
      }
  hs.d_prof = (double*)dalloc(c, box.size() * sizeof(double));
  if (!hs.d_prof) return fail(c, MM_ENOMEM, "hard source allocation failed");
  HIPCHECK(c, hipMemcpy(hs.d_prof, box.data(), box.size() * sizeof(double), hipMemcpyHostToDevice));
  c->hard.push_back(hs);
  if (field >= 3) {
    // the source's tiles leave the fused far pass: rebuild the tile lists
    void* old[7] = {c->d_tl_all, c->d_tl_near, c->d_tl_far, c->d_far, c->d_tl_pml, c->d_tl_all2, c->d_tl_all1};
    for (void* q : old)
      if (q) dfree(c, q);
    mm_status ts = build_tiles(c);
    if (!ts) ts = flux_mask(c);
    if (ts) return ts;
  }
  return MM_OK;
}

}  // namespace

mm_status mm_add_hard_source(mm_ctx* c, const mm_hard_source* s) {
  if (!c || !s) return MM_EINVAL;
  return add_hard(c, s->field, s->profile, s->f0, s->Tp, s->t0);
}

mm_status mm_add_surface_current(mm_ctx* c, const mm_surface_current* s) {
  if (!c || !s) return MM_EINVAL;
  const int axis = s->axis, comp = s->comp, side = s->side;
  if (axis < 0 || axis > 2 || comp < 0 || comp > 2 || comp == axis || (side != 0 && side != 1) || !s->profile)
    return fail(c, MM_EINVAL, "bad surface current (axis %d, side %d, comp %d)", axis, side, comp);
  if (c->per >> axis & 1) return fail(c, MM_EINVAL, "a surface current needs a PEC wall (axis %d is periodic)", axis);
  const int h = 3 - axis - comp;
  // H_t = J_s x n with n = +e_axis at the low wall and -e_axis at the high
  // wall: H_h = J * eps(comp, axis, h) * (side ? -1 : +1)
  const int eps = ((comp + 1) % 3 == axis) ? 1 : -1;
  const double sign = side ? -eps : eps;
  int je[3], he[3];
  field_extent(c, comp, je);
  field_extent(c, 3 + h, he);
  std::vector<double> H((size_t)he[0] * he[1] * he[2], 0.0);
  const int wall = side ? ncell(c, axis) : 0;       // the wall's node index along axis
  const int first = side ? ncell(c, axis) - 1 : 0;  // the cell beside it
  for (int k = 0; k < je[2]; ++k)
    for (int j = 0; j < je[1]; ++j)
      for (int i = 0; i < je[0]; ++i) {
        const int p[3] = {i, j, k};
        if (p[axis] != wall) continue;
        int q[3] = {i, j, k};
        q[axis] = first;
        const double v = s->profile[(size_t)i + (size_t)je[0] * ((size_t)j + (size_t)je[1] * k)];
        H[(size_t)q[0] + (size_t)he[0] * ((size_t)q[1] + (size_t)he[1] * q[2])] = sign * v;
      }
  return add_hard(c, 3 + h, H.data(), s->f0, s->Tp, s->t0);
}

mm_status mm_add_probe(mm_ctx* c, const mm_probe_desc* d, int32_t* id) {
  if (!c || !d) return MM_EINVAL;
  if (c->step > 0 || c->probes_frozen) return fail(c, MM_ESTATE, "probes must be added before the first step");
  ProbeRec r;
  r.d = *d;
  std::memset(&r.pp, 0, sizeof r.pp);
  if (d->kind == 1) {
    const bool pxp = c->per & 1;
    if (pxp ? (d->i < 0 || d->i >= c->nx) : (d->i < 1 || d->i >= c->nx))
      return fail(c, MM_EINVAL, "flux plane must be an interior x node");
  } else if (d->kind == 0) {
    if (d->field < 0 || d->field > 17) return fail(c, MM_EINVAL, "bad probe field");
    int ext[3];
    field_extent(c, d->field, ext);
    if (d->i < 0 || d->j < 0 || d->k < 0 || d->i >= ext[0] || d->j >= ext[1] || d->k >= ext[2])
      return fail(c, MM_EINVAL, "probe index outside the field extent");
    const int pi = (int)pidx(c, d->i, d->j, d->k);
    r.pp.fam = -1;
    r.pp.pi = d->i;
    r.pp.pj = d->j;
    r.pp.pk = d->k;
    if (d->field >= 3 && d->field < 6) r.pp.fam = d->field - 3;
    if (d->field >= 15) r.pp.fam = d->field - 15;
    if (d->field < 6) {
      r.pp.h = d->field < 3 ? c->E[d->field] : c->H[d->field - 3];
      r.pp.ih = pi;
      r.pp.ch = 1.0;
    } else {
      const int f = d->field < 15 ? (d->field - 6) / 3 : d->field - 15;
      int m = -1;
      for (size_t q = 0; q < c->h_idx.size(); ++q)
        if (c->h_fam[q] == f && c->h_idx[q] == pi) { m = (int)q; break; }
      if (d->field < 15) {
        const int comp = (d->field - 6) % 3;
        if (m >= 0) {
          r.pp.mcomp = c->d_M[comp];
          r.pp.im = m;
          r.pp.cm = 1.0;
        }
      } else {
        r.pp.h = c->H[f];
        r.pp.ih = pi;
        if (m >= 0) {
          r.pp.ch = mmk::kMu0;
          r.pp.mcomp = c->d_M[f];
          r.pp.im = m;
          r.pp.cm = mmk::kMu0;
        } else {
          // mu_f from the two cells beside the face (clamped at PEC walls)
          double mu = 1.0;
          if (c->mu) {
            std::vector<double> tmp(c->nelem);
            if (c->esz == 8) {
              HIPCHECK(c, hipMemcpy(tmp.data(), c->mu, c->nelem * 8, hipMemcpyDeviceToHost));
            } else {
              std::vector<float> tf(c->nelem);
              HIPCHECK(c, hipMemcpy(tf.data(), c->mu, c->nelem * 4, hipMemcpyDeviceToHost));
              for (size_t q = 0; q < c->nelem; ++q) tmp[q] = tf[q];
            }
            int qa[3] = {d->i, d->j, d->k}, qb[3] = {d->i, d->j, d->k};
            qa[f] -= 1;
            const int nf = ncell(c, f);
            if (qa[f] < 0) qa[f] = (c->per >> f & 1) ? nf - 1 : 0;
            if (qb[f] >= nf) qb[f] = nf - 1;
            mu = 0.5 * (tmp[pidx(c, qa[0], qa[1], qa[2])] + tmp[pidx(c, qb[0], qb[1], qb[2])]);
          }
          r.pp.ch = mmk::kMu0 * mu;
        }
      }
    }
  } else {
    return fail(c, MM_EINVAL, "bad probe kind");
  }
  c->probes.push_back(r);
  if (id) *id = (int32_t)(c->probes.size() - 1);
  return MM_OK;
}

mm_status mm_probe(mm_ctx* c, int32_t id, double* out, size_t cap, size_t* n_written, double* sum) {
  if (!c) return MM_EINVAL;
  if (id < 0 || (size_t)id >= c->probes.size()) return fail(c, MM_EINVAL, "bad probe id");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const size_t n = (size_t)c->step;
  if (n_written) *n_written = n;
  if (out && n && c->d_series) {
    const size_t m = std::min(cap, n);
    HIPCHECK(c, hipMemcpy(out, c->d_series + (size_t)id * c->series_cap, m * sizeof(double), hipMemcpyDeviceToHost));
  }
  if (sum) {
    *sum = 0.0;
    if (c->d_sums) HIPCHECK(c, hipMemcpy(sum, c->d_sums + id, sizeof(double), hipMemcpyDeviceToHost));
  }
  mm_status s = read_sticky(c);
  if (s) return s;
  return take_sticky(c);
}

mm_status mm_get_field(mm_ctx* c, int32_t field, double* dst) {
  if (!c || !dst) return MM_EINVAL;
  if (field < 0 || field > 17) return fail(c, MM_EINVAL, "bad field id");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  int ext[3];
  field_extent(c, field, ext);
  const size_t n = (size_t)ext[0] * ext[1] * ext[2];
  std::fill(dst, dst + n, 0.0);
  auto out_at = [&](int i, int j, int k) -> double& {
    return dst[(size_t)i + (size_t)ext[0] * ((size_t)j + (size_t)ext[1] * k)];
  };
  std::vector<double> fld;
  auto fetch = [&](void* p) -> mm_status {
    fld.assign(c->nelem, 0.0);
    if (c->esz == 8) {
      HIPCHECK(c, hipMemcpy(fld.data(), p, c->nelem * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tf(c->nelem);
      HIPCHECK(c, hipMemcpy(tf.data(), p, c->nelem * 4, hipMemcpyDeviceToHost));
      for (size_t q = 0; q < c->nelem; ++q) fld[q] = tf[q];
    }
    return MM_OK;
  };
  const size_t ntot = c->h_idx.size();
  std::vector<double> mc;
  auto fetch_m = [&](int comp) -> mm_status {
    mc.assign(ntot, 0.0);
    if (ntot) HIPCHECK(c, hipMemcpy(mc.data(), c->d_M[comp], ntot * sizeof(double), hipMemcpyDeviceToHost));
    return MM_OK;
  };
  mm_status s;
  if (field < 6) {
    s = fetch(field < 3 ? c->E[field] : c->H[field - 3]);
    if (s) return s;
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) out_at(i, j, k) = fld[pidx(c, i, j, k)];
  } else if (field < 15) {
    const int f = (field - 6) / 3, comp = (field - 6) % 3;
    s = fetch_m(comp);
    if (s) return s;
    for (size_t q = 0; q < ntot; ++q) {
      if (c->h_fam[q] != f) continue;
      const int pi = c->h_idx[q];
      const int k = pi / (c->px * c->py), r = pi - k * c->px * c->py, j = r / c->px, i = r - j * c->px;
      out_at(i, j, k) = mc[q];
    }
  } else {
    const int f = field - 15;
    s = fetch(c->H[f]);
    if (s) return s;
    std::vector<double> mu;
    if (c->mu) {
      std::vector<double> keep = fld;
      s = fetch(c->mu);
      if (s) return s;
      mu = fld;
      fld = keep;
    }
    const int nf = ncell(c, f);
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) {
          double muf = 1.0;
          if (c->mu) {
            int qa[3] = {i, j, k}, qb[3] = {i, j, k};
            qa[f] -= 1;
            if (qa[f] < 0) qa[f] = (c->per >> f & 1) ? nf - 1 : 0;
            if (qb[f] >= nf) qb[f] = nf - 1;
            muf = 0.5 * (mu[pidx(c, qa[0], qa[1], qa[2])] + mu[pidx(c, qb[0], qb[1], qb[2])]);
          }
          out_at(i, j, k) = mmk::kMu0 * muf * fld[pidx(c, i, j, k)];
        }
    s = fetch_m(f);
    if (s) return s;
    for (size_t q = 0; q < ntot; ++q) {
      if (c->h_fam[q] != f) continue;
      const int pi = c->h_idx[q];
      const int k = pi / (c->px * c->py), r = pi - k * c->px * c->py, j = r / c->px, i = r - j * c->px;
      out_at(i, j, k) = mmk::kMu0 * (fld[pi] + mc[q]);
    }
  }
  s = read_sticky(c);
  if (s) return s;
  return take_sticky(c);
}

mm_status mm_set_field(mm_ctx* c, int32_t field, const double* src) {
  if (!c || !src) return MM_EINVAL;
  if (field < 0 || field > 5) return fail(c, MM_EINVAL, "only E and H components can be set");
  int ext[3];
  field_extent(c, field, ext);
  void* p = field < 3 ? c->E[field] : c->H[field - 3];
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  if (c->esz == 8) {
    std::vector<double> h(c->nelem, 0.0);
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i)
          if (entry_interior(c, field, i, j, k))
            h[pidx(c, i, j, k)] = src[(size_t)i + (size_t)ext[0] * ((size_t)j + (size_t)ext[1] * k)];
    HIPCHECK(c, hipMemcpy(p, h.data(), c->nelem * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> h(c->nelem, 0.0f);
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i)
          if (entry_interior(c, field, i, j, k))
            h[pidx(c, i, j, k)] = (float)src[(size_t)i + (size_t)ext[0] * ((size_t)j + (size_t)ext[1] * k)];
    HIPCHECK(c, hipMemcpy(p, h.data(), c->nelem * 4, hipMemcpyHostToDevice));
  }
  return MM_OK;
}

namespace {

// Copy between the padded device array of E/H component `field` and a dense
// device buffer of its staggered extent (to_dense: padded -> dense).
mm_status copy_dense(mm_ctx* c, int field, void* dense, bool to_dense) {
  int ext[3];
  field_extent(c, field, ext);
  void* p = field < 3 ? c->E[field] : c->H[field - 3];
  hipMemcpy3DParms q;
  std::memset(&q, 0, sizeof q);
  const hipPitchedPtr padded = make_hipPitchedPtr(p, (size_t)c->px * c->esz, (size_t)c->px, (size_t)c->py);
  const hipPitchedPtr flat = make_hipPitchedPtr(dense, (size_t)ext[0] * c->esz, (size_t)ext[0], (size_t)ext[1]);
  q.srcPtr = to_dense ? padded : flat;
  q.dstPtr = to_dense ? flat : padded;
  q.extent = make_hipExtent((size_t)ext[0] * c->esz, (size_t)ext[1], (size_t)ext[2]);
  q.kind = hipMemcpyDeviceToDevice;
  HIPCHECK(c, hipMemcpy3DAsync(&q, c->stream));
  return MM_OK;
}

}  // namespace

mm_status mm_get_field_device(mm_ctx* c, int32_t field, void* dst) {
  if (!c || !dst) return MM_EINVAL;
  if (field < 0 || field > 5) return fail(c, MM_EINVAL, "device access covers E and H components only");
  return copy_dense(c, field, dst, true);
}

mm_status mm_set_field_device(mm_ctx* c, int32_t field, const void* src) {
  if (!c || !src) return MM_EINVAL;
  if (field < 0 || field > 5) return fail(c, MM_EINVAL, "only E and H components can be set");
  mm_status s = copy_dense(c, field, const_cast<void*>(src), false);
  if (s) return s;
  // PEC walls: E_c is pinned where an index along a != c is 0 or n_a, H_f
  // where its index along f is 0 or n_f
  char* p = (char*)(field < 3 ? c->E[field] : c->H[field - 3]);
  int ext[3];
  field_extent(c, field, ext);
  const size_t es = c->esz, row = (size_t)c->px * es, plane = row * c->py;
  for (int a = 0; a < 3; ++a) {
    const bool wall_axis = field < 3 ? a != field : a == field - 3;
    if (!wall_axis || (c->per >> a & 1)) continue;
    for (int v : {0, ncell(c, a)}) {
      if (a == 2) {
        HIPCHECK(c, hipMemsetAsync(p + (size_t)v * plane, 0, plane, c->stream));
      } else if (a == 1) {
        HIPCHECK(c, hipMemset2DAsync(p + (size_t)v * row, plane, 0, row, (size_t)ext[2], c->stream));
      } else {
        HIPCHECK(c, hipMemset2DAsync(p + (size_t)v * es, row, 0, es, (size_t)c->py * ext[2], c->stream));
      }
    }
  }
  return MM_OK;
}

mm_status mm_stats(mm_ctx* c, int32_t* iters, size_t cap, size_t* n) {
  if (!c) return MM_EINVAL;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const size_t tot = (size_t)c->substep;
  if (n) *n = tot;
  if (iters && tot) {
    const size_t m = std::min(cap, tot);
    if (c->nmag > 0) {
      HIPCHECK(c, hipMemcpy(iters, c->d_iters, m * sizeof(int), hipMemcpyDeviceToHost));
    } else {
      for (size_t q = 0; q < m; ++q) iters[q] = c->fixed_iter > 0 ? c->fixed_iter : 1;
    }
  }
  mm_status s = read_sticky(c);
  if (s) return s;
  return take_sticky(c);
}

mm_status mm_sync(mm_ctx* c) {
  if (!c) return MM_EINVAL;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  mm_status s = read_sticky(c);
  if (s) return s;
  return take_sticky(c);
}

mm_status mm_info(const mm_ctx* c, int64_t out[8]) {
  if (!c || !out) return MM_EINVAL;
  out[0] = c->nmag;
  out[1] = c->nwall;
  out[2] = c->nsrc;
  out[3] = c->px;
  out[4] = c->py;
  out[5] = c->pz;
  out[6] = (int64_t)c->esz;
  out[7] = (int64_t)c->dev_bytes;
  return MM_OK;
}

mm_status mm_layout(const mm_ctx* c, int64_t out[8]) {
  if (!c || !out) return MM_EINVAL;
  out[0] = c->n_all;
  out[1] = c->n_near;
  out[2] = c->n_far;
  out[3] = c->cells_near;
  out[4] = c->cells_far;
  out[5] = c->tkc;
  out[6] = c->nmat;
  out[7] = c->n_pml;
  return MM_OK;
}

mm_status mm_adjoint_enable(mm_ctx* c, int32_t checkpoint_every, int32_t inner_every) {
  if (!c) return MM_EINVAL;
  if (!c->hard.empty()) return fail(c, MM_EINVAL, "the adjoint does not cover hard sources");
  if (checkpoint_every < 1) return fail(c, MM_EINVAL, "checkpoint_every must be >= 1");
  if (inner_every < 0 || inner_every > checkpoint_every)
    return fail(c, MM_EINVAL, "inner_every must be in [0, checkpoint_every]");
  if (c->step != 0) return fail(c, MM_ESTATE, "the adjoint must be enabled before the first step");
  if (c->mu) return fail(c, MM_EINVAL, "the adjoint supports mu_r = 1 only");
  if (c->scheme != 2) return fail(c, MM_EINVAL, "the adjoint supports the second-order scheme only");
  if (c->has_pml) return fail(c, MM_EINVAL, "the adjoint does not support an open boundary");
  c->ckpt_every = checkpoint_every;
  c->ckpt_inner = inner_every;
  return MM_OK;
}

mm_status mm_adjoint(mm_ctx* c, int32_t probe_id, double* grad_eps_r, double* grad_Ms) {
  if (!c || !grad_eps_r || !grad_Ms) return MM_EINVAL;
  if (c->ckpt_every <= 0) return fail(c, MM_ESTATE, "mm_adjoint_enable was not called before stepping");
  if (probe_id < 0 || (size_t)probe_id >= c->probes.size() || c->probes[probe_id].d.kind != 1)
    return fail(c, MM_EINVAL, "the loss probe must be a flux probe");
  if (c->step == 0) return fail(c, MM_ESTATE, "no steps to differentiate");
  mm_status s = mm_sync(c);
  if (s) return s;
  const int i0 = c->probes[probe_id].d.i;
  s = c->prec == MM_FP32 ? adjoint_run<float>(c, i0, grad_eps_r, grad_Ms)
                         : adjoint_run<double>(c, i0, grad_eps_r, grad_Ms);
  if (s) return s;
  s = read_sticky(c);
  if (s) return s;
  return take_sticky(c);
}

mm_status mm_profile(mm_ctx* c, int32_t enable) {
  if (!c) return MM_EINVAL;
  c->prof = enable != 0;
  return MM_OK;
}

mm_status mm_profile_read(mm_ctx* c, double ms[8], int64_t counts[8]) {
  if (!c || !ms || !counts) return MM_EINVAL;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  for (int q = 0; q < 8; ++q) {
    ms[q] = 0.0;
    counts[q] = 0;
  }
  for (size_t q = 0; q < c->ev_used; ++q) {
    float t = 0.f;
    HIPCHECK(c, hipEventElapsedTime(&t, c->ev_pool[q].first, c->ev_pool[q].second));
    ms[c->ev_class[q]] += t;
    counts[c->ev_class[q]] += 1;
  }
  c->ev_used = 0;
  return MM_OK;
}

const char* mm_last_error(const mm_ctx* c) { return c ? c->err.c_str() : "null context"; }

void mm_destroy(mm_ctx* c) {
  if (!c) return;
  release(c);
  delete c;
}

}  // extern "C"
