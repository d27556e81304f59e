// Host side of the adjoint (included by mm.hip inside its anonymous
// namespace, after the forward runtime).
//
// Forward: with mm_adjoint_enable(c, K), mm_step saves the state (E, H, M)
// at every step index that is a multiple of K.
// mm_adjoint: for each K-step segment, last first, restore its checkpoint
// and recompute the segment, storing per step E^{n+1} (the out-of-place E
// update writes it there), M^n, M^{n+1/2}, the H iterates of both sub-steps,
// H^n and H^{n+1/2} on the faces the magnetic rows touch only, and the flux
// plane's level n+1 H values; then reverse the steps (flux seed at n+1,
// Step 3, Step 2, Step 1) with the kernels of adjoint.h.  On large grids the
// far tiles lag half a step in that recompute, as in a forward run.
// Two-level (inner spacing K2 < K): the segment is first recomputed once,
// saving the state every K2 steps, and then reversed K2 steps at a time,
// so only K2 steps of per-step storage are held.
// Finally map the edge-eps and face-Ms cotangents to the cell maps on the
// host and put the final state back.

struct AdjWork {
  int K = 0;                   // outer checkpoint spacing (steps)
  int K2 = 0;                  // inner spacing: steps stored per reversed span (K2 <= K)
  int cap = 0;                 // iterate-log slots per sub-step
  std::vector<void*> ick;      // inner checkpoints of the current outer segment (two-level)
  void* Eb[3] = {};
  void* Hb[3] = {};
  void* Xb[3] = {};
  void* Gb[3] = {};
  void* W[3] = {};
  double* Q[9] = {};
  double** dQ = nullptr;
  double* epsb[3] = {};
  // per step j of a span: sE[j] = E^{n+1} (written there by the out-of-place
  // E update; E^n of step 0 stays in the live E); sHc, sHh: H^n, H^{n+1/2}
  // on the touched faces only
  // (sHc, sHh in the order of the touched-face list); sP: the flux seed's H
  // values of the plane at level n+1 (see plane_store)
  std::vector<void*> sE, sHc, sHh, sP;
  std::vector<double*> sM, sMh, slog;
  void* Hsc[3] = {};                 // full-size H scratch the compact levels are scattered into
  int cap_p = -1;                    // the loss plane's index in the flux-plane capture
  double *b[3] = {}, *d[3] = {}, *hes[3] = {}, *bb[3] = {}, *db[3] = {}, *Mb[3] = {};
  double *qb = nullptr, *hbit = nullptr, *msf_b = nullptr, *aoms_b = nullptr;
  int* tidx = nullptr;
  unsigned char* tfam = nullptr;
  int* tmag = nullptr;
  int nt = 0;
  void* fin = nullptr;
};

size_t state_bytes(const mm_ctx* c) {
  return 6 * c->nelem * c->esz + 3 * (c->h_idx.size() ? c->h_idx.size() : 1) * sizeof(double);
}

// Copies (dst[q] <- src[q], bytes[q], multiples of 8) in one launch.
struct CopyList {
  int n = 0;
  const void* src[mmk::kCopyMax];
  void* dst[mmk::kCopyMax];
  size_t bytes[mmk::kCopyMax];
  void add(const void* s, void* d, size_t b) {
    src[n] = s;
    dst[n] = d;
    bytes[n] = b;
    ++n;
  }
};

mm_status run_copies(mm_ctx* c, const CopyList& L) {
  if (L.n == 0) return MM_OK;
  mmk::CopyBatch b;
  std::memset(&b, 0, sizeof b);
  size_t most = 0;
  for (int q = 0; q < L.n; ++q) {
    b.src[q] = (const unsigned long long*)L.src[q];
    b.dst[q] = (unsigned long long*)L.dst[q];
    b.words[q] = L.bytes[q] / 8;
    most = std::max(most, L.bytes[q] / 8);
  }
  const unsigned gx = (unsigned)std::max<size_t>(1, std::min<size_t>((most + 1023) / 1024, 2048));
  hipLaunchKernelGGL(mmk::copy_batch, dim3(gx, L.n), dim3(256), 0, c->stream, b);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// E, H and M to (save) or from a block laid out as E0 E1 E2 H0 H1 H2
// (nelem * esz each), M0 M1 M2 (ntot doubles each), added to a copy list.
void add_state(const mm_ctx* c, CopyList& L, void* blk, bool save) {
  const size_t fb = c->nelem * c->esz;
  const size_t ntot = c->h_idx.size();
  char* p = (char*)blk;
  for (int a = 0; a < 3; ++a) {
    void* e = p + a * fb;
    void* h = p + (3 + a) * fb;
    L.add(save ? c->E[a] : e, save ? e : c->E[a], fb);
    L.add(save ? c->H[a] : h, save ? h : c->H[a], fb);
  }
  if (ntot)
    for (int a = 0; a < 3; ++a) {
      void* m = p + 6 * fb + a * ntot * sizeof(double);
      L.add(save ? (void*)c->d_M[a] : m, save ? m : (void*)c->d_M[a], ntot * sizeof(double));
    }
}

// state block layout: see add_state
mm_status copy_state(mm_ctx* c, void* blk, bool save) {
  CopyList L;
  add_state(c, L, blk, save);
  return run_copies(c, L);
}

mm_status save_checkpoint(mm_ctx* c, size_t idx) {
  while (c->ckpts.size() <= idx) {
    void* blk = dalloc(c, state_bytes(c));
    if (!blk) return fail(c, MM_ENOMEM, "checkpoint allocation failed");
    c->ckpts.push_back(blk);
  }
  return copy_state(c, c->ckpts[idx], true);
}

// 3 field arrays (E or H) to / from a packed block of 3 arrays
void add3(const mm_ctx* c, CopyList& L, void* blk, void* const* arr, bool save) {
  const size_t fb = c->nelem * c->esz;
  for (int a = 0; a < 3; ++a) {
    void* q = (char*)blk + a * fb;
    L.add(save ? arr[a] : q, save ? q : arr[a], fb);
  }
}

void addM(const mm_ctx* c, CopyList& L, double* blk, bool save) {
  const size_t ntot = c->h_idx.size();
  for (int a = 0; a < 3 && ntot; ++a)
    L.add(save ? (void*)c->d_M[a] : (void*)(blk + a * ntot), save ? (void*)(blk + a * ntot) : (void*)c->d_M[a],
          ntot * sizeof(double));
}

// Faces that evolving magnetic faces read (themselves and their 8
// transverse neighbours), each once: the evolving faces first, entry t
// holding face t (compact index t), then the other faces they read (-1).
// Returns false if a neighbour falls outside the padded grid.
bool touched_faces(const mm_ctx* c, std::vector<int>& idx, std::vector<unsigned char>& fam, std::vector<int>& mag) {
  const size_t ne = c->nelem;
  std::vector<uint64_t> seen((3 * ne + 63) / 64, 0);   // one bit per (family, padded index)
  auto dn = [&](int i, int n, bool p) { return (p && i == 0) ? n - 1 : i - 1; };
  auto up = [&](int i, int n, bool p) { return (p && i == n - 1) ? 0 : i + 1; };
  const bool pxp = c->per & 1, pyp = c->per & 2, pzp = c->per & 4;
  bool ok = true;
  auto add = [&](int f, long long pi, int m) {
    if (pi < 0 || (size_t)pi >= ne) {
      ok = false;
      return;
    }
    const size_t key = (size_t)f * ne + (size_t)pi;
    uint64_t& word = seen[key >> 6];
    const uint64_t bit = 1ull << (key & 63);
    if (word & bit) return;
    word |= bit;
    idx.push_back((int)pi);
    fam.push_back((unsigned char)f);
    mag.push_back(m);
  };
  const size_t nm = (size_t)c->nmag;
  idx.reserve(4 * nm);
  fam.reserve(4 * nm);
  mag.reserve(4 * nm);
  for (int t = 0; t < c->nmag; ++t) add(c->h_fam[t], c->h_idx[t], t);
  auto P = [&](int a, int b2, int d2) {
    return a < 0 || b2 < 0 || d2 < 0 ? -1ll : (long long)pidx(c, a, b2, d2);
  };
  for (int t = 0; t < c->nmag; ++t) {
    const int pi = c->h_idx[t], f = c->h_fam[t];
    const int k = pi / (c->px * c->py), rr = pi - k * c->px * c->py, j = rr / c->px, i = rr - j * c->px;
    if (f == 0) {
      const int im = dn(i, c->nx, pxp), jp = up(j, c->ny, pyp), kp = up(k, c->nz, pzp);
      add(1, P(im, j, k), -1); add(1, P(i, j, k), -1); add(1, P(im, jp, k), -1); add(1, P(i, jp, k), -1);
      add(2, P(im, j, k), -1); add(2, P(i, j, k), -1); add(2, P(im, j, kp), -1); add(2, P(i, j, kp), -1);
    } else if (f == 1) {
      const int jm = dn(j, c->ny, pyp), ip = up(i, c->nx, pxp), kp = up(k, c->nz, pzp);
      add(0, P(i, jm, k), -1); add(0, P(i, j, k), -1); add(0, P(ip, jm, k), -1); add(0, P(ip, j, k), -1);
      add(2, P(i, jm, k), -1); add(2, P(i, j, k), -1); add(2, P(i, jm, kp), -1); add(2, P(i, j, kp), -1);
    } else {
      const int km = dn(k, c->nz, pzp), ip = up(i, c->nx, pxp), jp = up(j, c->ny, pyp);
      add(0, P(i, j, km), -1); add(0, P(i, j, k), -1); add(0, P(ip, j, km), -1); add(0, P(ip, j, k), -1);
      add(1, P(i, j, km), -1); add(1, P(i, j, k), -1); add(1, P(i, jp, km), -1); add(1, P(i, jp, k), -1);
    }
  }
  return ok;
}

// Largest iteration count of the sub-steps run so far (the recompute repeats
// them exactly), at most 16: the number of iterate-log slots needed.
mm_status iterate_slots(mm_ctx* c, int& slots) {
  int maxit = 1;
  if (c->nmag > 0 && c->step > 0) {
    std::vector<int> it(2 * (size_t)c->step);
    HIPCHECK(c, hipMemcpy(it.data(), c->d_iters, it.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (int v : it) maxit = std::max(maxit, v);
  }
  slots = std::min(maxit, 16);
  return MM_OK;
}

mm_status adj_alloc(mm_ctx* c) {
  int slots = 1;
  mm_status st = iterate_slots(c, slots);
  if (st) return st;
  if (c->adjw) {   // allocated by an earlier call: grow the iterate logs if needed
    AdjWork* w = c->adjw;
    if (w->cap >= slots) {
      c->hlog_cap = w->cap;
      return MM_OK;
    }
    const size_t nm = (size_t)std::max(c->nmag, 1);
    for (auto& lg : w->slog) {
      dfree(c, lg);
      lg = (double*)dalloc(c, 2 * (size_t)slots * nm * 8);
      if (!lg) return fail(c, MM_ENOMEM, "adjoint segment storage allocation failed");
    }
    w->cap = slots;
    c->hlog_cap = slots;
    return MM_OK;
  }
  AdjWork* w = new AdjWork();
  c->adjw = w;
  w->K = c->ckpt_every;
  w->K2 = c->ckpt_inner > 0 ? std::min(c->ckpt_inner, c->ckpt_every) : c->ckpt_every;
  w->cap = slots;
  c->hlog_cap = w->cap;
  const size_t fb = c->nelem * c->esz, fd = c->nelem * sizeof(double);
  auto need = [&](void* p) { return p != nullptr; };
  for (int a = 0; a < 3; ++a) {
    w->Eb[a] = dalloc(c, fb);
    w->Hb[a] = dalloc(c, fb);
    w->Xb[a] = dalloc(c, fb);
    w->Gb[a] = dalloc(c, fb);
    w->W[a] = dalloc(c, fb);
    w->epsb[a] = (double*)dalloc(c, fd);
    if (!need(w->Eb[a]) || !need(w->Hb[a]) || !need(w->Xb[a]) || !need(w->Gb[a]) || !need(w->W[a]) ||
        !need(w->epsb[a]))
      return fail(c, MM_ENOMEM, "adjoint work allocation failed");
    for (void* p : {w->Xb[a], w->Gb[a], w->W[a]}) HIPCHECK(c, hipMemsetAsync(p, 0, fb, c->stream));
  }
  const size_t nm = (size_t)std::max(c->nmag, 1);
  const size_t ntot = std::max<size_t>(c->h_idx.size(), 1);
  if (c->nmag > 0) {
    for (int q = 0; q < 9; ++q) {
      w->Q[q] = (double*)dalloc(c, fd);
      if (!w->Q[q]) return fail(c, MM_ENOMEM, "adjoint work allocation failed");
      HIPCHECK(c, hipMemsetAsync(w->Q[q], 0, fd, c->stream));
    }
    w->dQ = (double**)dalloc(c, 9 * sizeof(double*));
    if (!w->dQ) return fail(c, MM_ENOMEM, "adjoint work allocation failed");
    HIPCHECK(c, hipMemcpy(w->dQ, w->Q, 9 * sizeof(double*), hipMemcpyHostToDevice));
    for (int a = 0; a < 3; ++a) {
      w->b[a] = (double*)dalloc(c, nm * 8);
      w->d[a] = (double*)dalloc(c, nm * 8);
      w->hes[a] = (double*)dalloc(c, nm * 8);
      w->bb[a] = (double*)dalloc(c, nm * 8);
      w->db[a] = (double*)dalloc(c, nm * 8);
      w->Mb[a] = (double*)dalloc(c, ntot * 8);
      if (!w->b[a] || !w->d[a] || !w->hes[a] || !w->bb[a] || !w->db[a] || !w->Mb[a])
        return fail(c, MM_ENOMEM, "adjoint work allocation failed");
    }
    w->qb = (double*)dalloc(c, nm * 8);
    w->hbit = (double*)dalloc(c, nm * 8);
    w->msf_b = (double*)dalloc(c, nm * 8);
    w->aoms_b = (double*)dalloc(c, nm * 8);
    if (!w->qb || !w->hbit || !w->msf_b || !w->aoms_b) return fail(c, MM_ENOMEM, "adjoint work allocation failed");
    std::vector<int> ti, tm;
    std::vector<unsigned char> tf;
    if (!touched_faces(c, ti, tf, tm))
      return fail(c, MM_ESTATE, "adjoint: a magnetic face's neighbour lies outside the grid");
    w->nt = (int)ti.size();
    w->tidx = (int*)dalloc(c, ti.size() * 4);
    w->tfam = (unsigned char*)dalloc(c, tf.size());
    w->tmag = (int*)dalloc(c, tm.size() * 4);
    if (!w->tidx || !w->tfam || !w->tmag) return fail(c, MM_ENOMEM, "adjoint work allocation failed");
    HIPCHECK(c, hipMemcpy(w->tidx, ti.data(), ti.size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(w->tfam, tf.data(), tf.size(), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(w->tmag, tm.data(), tm.size() * 4, hipMemcpyHostToDevice));
  }
  for (void*& p : w->Hsc) {
    p = dalloc(c, 3 * fb);
    if (!p) return fail(c, MM_ENOMEM, "adjoint work allocation failed");
  }
  for (int q = 1; q * w->K2 < w->K; ++q) {
    void* blk = dalloc(c, state_bytes(c));
    if (!blk) return fail(c, MM_ENOMEM, "inner checkpoint allocation failed");
    w->ick.push_back(blk);
  }
  for (int j = 0; j < w->K2; ++j) {
    void* e = dalloc(c, 3 * fb);
    void* h = dalloc(c, (size_t)std::max(w->nt, 1) * c->esz);
    void* hh = dalloc(c, (size_t)std::max(w->nt, 1) * c->esz);
    void* pl = dalloc(c, (size_t)4 * nodes(c, 1) * nodes(c, 2) * c->esz);
    if (!pl) return fail(c, MM_ENOMEM, "adjoint segment storage allocation failed");
    w->sP.push_back(pl);
    double* m = (double*)dalloc(c, 3 * ntot * 8);
    double* mh = (double*)dalloc(c, 3 * ntot * 8);
    double* lg = (double*)dalloc(c, 2 * (size_t)w->cap * nm * 8);
    if (!e || !h || !hh || !m || !mh || !lg) return fail(c, MM_ENOMEM, "adjoint segment storage allocation failed");
    w->sE.push_back(e);
    w->sHc.push_back(h);
    w->sHh.push_back(hh);
    w->sM.push_back(m);
    w->sMh.push_back(mh);
    w->slog.push_back(lg);
  }
  w->fin = dalloc(c, state_bytes(c));
  if (!w->fin) return fail(c, MM_ENOMEM, "adjoint work allocation failed");
  return MM_OK;
}

mmk::AdjMag make_adjmag(const mm_ctx* c, const double* Ms0blk, const double* log) {
  const AdjWork& w = *c->adjw;
  const size_t ntot = c->h_idx.size();
  mmk::AdjMag a;
  a.idx = c->d_idx;
  a.nbm = c->d_nbm;
  a.Ms = c->d_Ms;
  a.kap = c->d_kap;
  a.aoms = c->d_aoms;
  for (int q = 0; q < 3; ++q) {
    a.Ms0[q] = Ms0blk + q * ntot;
    a.b[q] = w.b[q];
    a.d[q] = w.d[q];
    a.hes[q] = w.hes[q];
    a.bb[q] = w.bb[q];
    a.db[q] = w.db[q];
    a.Mb[q] = w.Mb[q];
  }
  a.hlog = log;
  a.qb = w.qb;
  a.hbit = w.hbit;
  a.msf_b = w.msf_b;
  a.aoms_b = w.aoms_b;
  a.off1 = c->off1;
  a.off2 = c->off2;
  a.n = c->nmag;
  return a;
}

template <typename T>
T* arr3(const void* blk, const mm_ctx* c, int a) {
  return (T*)((char*)blk + (size_t)a * c->nelem * c->esz);
}

// Reverse of one H-M sub-step whose input was (Hs, Ms0), output H (Ho),
// iterates `log` and count R.  With defer, it stops before the curl
// transpose: the caller runs it (inside adj_e_coef) and then adj_face_finish.
template <typename T>
mm_status adj_face_finish(mm_ctx* c);

template <typename T>
mm_status adj_substep(mm_ctx* c, T* const* Hs, const double* Ms0, T* const* Ho, const double* log, int R,
                      bool defer = false) {
  AdjWork& w = *c->adjw;
  Geo g = make_geo(c);
  T* Eb[3] = {(T*)w.Eb[0], (T*)w.Eb[1], (T*)w.Eb[2]};
  T* Hb[3] = {(T*)w.Hb[0], (T*)w.Hb[1], (T*)w.Hb[2]};
  T* Xb[3] = {(T*)w.Xb[0], (T*)w.Xb[1], (T*)w.Xb[2]};
  T* Gb[3] = {(T*)w.Gb[0], (T*)w.Gb[1], (T*)w.Gb[2]};
  T* Wv[3] = {(T*)w.W[0], (T*)w.W[1], (T*)w.W[2]};
  const double H0x = c->H0[0], H0y = c->H0[1], H0z = c->H0[2];
  if (c->nmag > 0) {
    mmk::AdjMag a = make_adjmag(c, Ms0, log);
    const int nb = (c->nmag + 255) / 256, tb = (w.nt + 255) / 256;
    const int gb = (std::max(w.nt, c->nmag) + 255) / 256;
    // iterate r reads iterate r - 1 of its magnetic neighbours from W: the
    // scatter of iterate r - 1 rides on the launch before iteration r (the
    // set-up for r = R, the gather of r + 1 otherwise)
    hipLaunchKernelGGL((mmk::adj_mag_prep<T>), dim3(nb), dim3(256), 0, c->stream, g, Hs[0], Hs[1], Hs[2], a, H0x,
                       H0y, H0z, Wv[0], Wv[1], Wv[2], R >= 2 ? R - 1 : 0);
    for (int r = R; r >= 1; --r) {
      hipLaunchKernelGGL((mmk::adj_mag_iter<T>), dim3(nb), dim3(256), 0, c->stream, g, a, Hs[0], Hs[1], Hs[2],
                         Ho[0], Ho[1], Ho[2], Wv[0], Wv[1], Wv[2], Hb[0], Hb[1], Hb[2], w.dQ, r, R, H0x, H0y,
                         H0z);
      hipLaunchKernelGGL((mmk::adj_gather<T>), dim3(r >= 2 ? gb : tb), dim3(256), 0, c->stream, g, w.tidx, w.tfam,
                         w.tmag, w.nt, w.dQ, a, Xb[0], Xb[1], Xb[2], Gb[0], Gb[1], Gb[2], r >= 2 ? 0 : 1, Wv[0],
                         Wv[1], Wv[2], r >= 3 ? r - 2 : 0, Hb[0], Hb[1], Hb[2], 0);
    }
    hipLaunchKernelGGL((mmk::adj_mag_inv<T>), dim3(nb), dim3(256), 0, c->stream, a, Xb[0], Xb[1], Xb[2], w.dQ);
    // with the face pass's first part (T = Hb + Xb on the touched faces)
    hipLaunchKernelGGL((mmk::adj_gather<T>), dim3(tb), dim3(256), 0, c->stream, g, w.tidx, w.tfam, w.tmag, w.nt,
                       w.dQ, a, Xb[0], Xb[1], Xb[2], Gb[0], Gb[1], Gb[2], 1, Wv[0], Wv[1], Wv[2], 0, Hb[0],
                       Hb[1], Hb[2], 1);
    HIPCHECK(c, hipGetLastError());
  } else if (w.nt > 0) {
    // the face pass's first part on its own (no magnetic rows ran)
    hipLaunchKernelGGL((mmk::adj_touch<T>), dim3((w.nt + 255) / 256), dim3(256), 0, c->stream, g, w.tidx, w.tfam,
                       w.nt, Hb[0], Hb[1], Hb[2], Xb[0], Xb[1], Xb[2], Gb[0], Gb[1], Gb[2], 0);
  }
  // then C = -(dt/2 mu0) T into curl E's transpose, Hb = T + Gb and the wall
  // faces cleared
  HIPCHECK(c, hipGetLastError());
  if (defer) return MM_OK;
  dim3 grid;
  const int kc = kchunk_for(c, grid);
  hipLaunchKernelGGL((mmk::add_curl_h<T>), grid, dim3(64, 4), 0, c->stream, g, Eb[0], Eb[1], Eb[2],
                     (const T*)Hb[0], (const T*)Hb[1], (const T*)Hb[2], -0.5 * c->dt / mmk::kMu0, kc);
  HIPCHECK(c, hipGetLastError());
  return adj_face_finish<T>(c);
}

// After the curl transpose: Hb = T + Gb on the touched faces (Xb, Gb
// cleared there) and the wall faces cleared.
template <typename T>
mm_status adj_face_finish(mm_ctx* c) {
  AdjWork& w = *c->adjw;
  const Geo g = make_geo(c);
  T* Hb[3] = {(T*)w.Hb[0], (T*)w.Hb[1], (T*)w.Hb[2]};
  T* Xb[3] = {(T*)w.Xb[0], (T*)w.Xb[1], (T*)w.Xb[2]};
  T* Gb[3] = {(T*)w.Gb[0], (T*)w.Gb[1], (T*)w.Gb[2]};
  const long long most = std::max({(long long)c->ny * c->nz, (long long)c->nx * c->nz, (long long)c->nx * c->ny,
                                   (long long)w.nt});
  hipLaunchKernelGGL((mmk::adj_face_end<T>), dim3((unsigned)((most + 255) / 256), 4), dim3(256), 0, c->stream, g,
                     w.tidx, w.tfam, w.nt, Hb[0], Hb[1], Hb[2], Xb[0], Xb[1], Xb[2], Gb[0], Gb[1], Gb[2]);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// Reverse of Step 2 of step c->step: En = E^n, E1 = E^{n+1}.  It opens
// with the curl transpose deferred by the Step 3 reverse before it (fused
// into adj_e_coef) and that reverse's face finish.
template <typename T>
mm_status adj_estep(mm_ctx* c, T* const* En, T* const* E1) {
  AdjWork& w = *c->adjw;
  Geo g = make_geo(c);
  dim3 grid;
  const int kc = kchunk_for(c, grid);
  T* Eb[3] = {(T*)w.Eb[0], (T*)w.Eb[1], (T*)w.Eb[2]};
  T* Hb[3] = {(T*)w.Hb[0], (T*)w.Hb[1], (T*)w.Hb[2]};
  T* Wv[3] = {(T*)w.W[0], (T*)w.W[1], (T*)w.W[2]};
  if (c->sig)
    hipLaunchKernelGGL((mmk::adj_e_coef<T, true>), grid, dim3(64, 4), 0, c->stream, g, Eb[0], Eb[1], Eb[2],
                       (const T*)En[0], (const T*)En[1], (const T*)En[2], (const T*)E1[0],
                       (const T*)E1[1], (const T*)E1[2], (const T*)c->eps, (const T*)c->sig, Wv[0], Wv[1],
                       Wv[2], w.epsb[0], w.epsb[1], w.epsb[2], (T)c->dt, (const T*)Hb[0], (const T*)Hb[1],
                       (const T*)Hb[2], -0.5 * c->dt / mmk::kMu0, kc);
  else
    hipLaunchKernelGGL((mmk::adj_e_coef<T, false>), grid, dim3(64, 4), 0, c->stream, g, Eb[0], Eb[1], Eb[2],
                       (const T*)En[0], (const T*)En[1], (const T*)En[2], (const T*)E1[0],
                       (const T*)E1[1], (const T*)E1[2], (const T*)c->eps, (const T*)c->sig, Wv[0], Wv[1],
                       Wv[2], w.epsb[0], w.epsb[1], w.epsb[2], (T)c->dt, (const T*)Hb[0], (const T*)Hb[1],
                       (const T*)Hb[2], -0.5 * c->dt / mmk::kMu0, kc);
  HIPCHECK(c, hipGetLastError());
  mm_status fs = adj_face_finish<T>(c);
  if (fs) return fs;
  // H_bar += curl E(W): the non-magnetic H kernel with coefficient -1
  hipLaunchKernelGGL((mmk::h_bulk<T, false, 1>), dim3(c->n_all), dim3(64, 4), 0, c->stream, g, Hb[0], Hb[1],
                     Hb[2], (const T*)Wv[0], (const T*)Wv[1], (const T*)Wv[2], (const T*)nullptr, (T)-1, (T)0,
                     tiles(c, c->d_tl_all));
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// The copies of L and, when out is set, the gather of H on the touched faces
// into `out`, in one launch.
template <typename T>
mm_status copies_and_gather(mm_ctx* c, const CopyList& L, T* out, const mmk::PlaneStore<T>* ps = nullptr) {
  AdjWork& w = *c->adjw;
  mmk::CopyBatch b;
  std::memset(&b, 0, sizeof b);
  size_t most = 0;
  for (int q = 0; q < L.n; ++q) {
    b.src[q] = (const unsigned long long*)L.src[q];
    b.dst[q] = (unsigned long long*)L.dst[q];
    b.words[q] = L.bytes[q] / 8;
    most = std::max(most, L.bytes[q] / 8);
  }
  const int ng = out ? w.nt : 0;
  mmk::PlaneStore<T> pst{};
  if (ps) pst = *ps;
  const size_t np = ps ? (size_t)pst.NY * pst.NZ : 0;
  const size_t bx = std::max({(most + 1023) / 1024, ((size_t)ng + 255) / 256, (np + 255) / 256});
  const unsigned gx = (unsigned)std::max<size_t>(1, std::min<size_t>(bx, 2048));
  const int gy = L.n + (ng > 0 ? 1 : 0) + (ps ? 1 : 0);
  if (gy == 0) return MM_OK;
  hipLaunchKernelGGL((mmk::copy_gather<T>), dim3(gx, gy), dim3(256), 0, c->stream, b, L.n, w.tidx, w.tfam, ng,
                     (const T*)c->H[0], (const T*)c->H[1], (const T*)c->H[2], out, pst);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// The live E pointers, put back when this goes out of scope.
struct KeepE {
  mm_ctx* c;
  void* E[3];
  explicit KeepE(mm_ctx* ctx) : c(ctx) {
    for (int a = 0; a < 3; ++a) E[a] = c->E[a];
  }
  ~KeepE() {
    for (int a = 0; a < 3; ++a) c->E[a] = E[a];
  }
};

// Steps [m0, m0 + len): restore the state saved at m0, recompute the span
// storing per step E^{n+1} (the E update writes it straight into sE[j] and
// the step goes on from there), M^n, M^{n+1/2}, the iterate logs and, at
// the list entries only, H^n and H^{n+1/2}; then reverse its steps, last
// first, into the cotangents.  E^{m0} stays in the live E arrays.
template <typename T>
mm_status reverse_span(mm_ctx* c, int i0, long m0, int len, void* start) {
  AdjWork& w = *c->adjw;
  const size_t lsub = (size_t)w.cap * std::max(c->nmag, 1);
  mm_status s = copy_state(c, start, false);
  if (s) return s;
  KeepE live(c);
  c->step = m0;
  c->substep = (int)(2 * m0);
  c->adj_recompute = true;
  // The far tiles lag half a step inside the span, as in a forward run: their
  // Step 3 of one step and Step 1 of the next go in one pass (h_far), which
  // also captures the flux plane's level n+1 values there.  The touched
  // faces all lie in near tiles, so the stores below see every level whole.
  // Lagging saves one pass over the far tiles per step and costs one launch,
  // so small grids (launch-bound) do without it.
  const long long far_cells = (long long)c->n_far * 64 * 4 * c->tkc;
  const bool lag_ok = c->n_far > 0 && c->d_fcap && c->tkc <= mmk::kCapPlanesZ && w.cap_p >= 0 &&
                      far_cells >= (1ll << 21);
  const Geo g = make_geo(c);
  const int NY = nodes(c, 1), NZ = nodes(c, 2);
  // the plane values of step j (level n+1) are stored by the first launch of
  // step j + 1, or on their own after the span's last step
  auto plane_args = [&](int jj, bool captured) {
    mmk::PlaneStore<T> a{};
    a.g = g;
    a.Hy = (const T*)c->H[1];
    a.Hz = (const T*)c->H[2];
    a.fc = flux_cap<T>(c, captured);
    a.p = w.cap_p;
    a.fmask = c->d_fmask;
    a.i0 = i0;
    a.NY = NY;
    a.NZ = NZ;
    a.out = jj >= 0 ? (T*)w.sP[jj] : nullptr;
    return a;
  };
  bool lagging = false;
  for (int j = 0; j < len; ++j) {
    const bool end = j == len - 1;
    {
      CopyList L;
      addM(c, L, w.sM[j], true);
      const mmk::PlaneStore<T> pa = plane_args(j - 1, lagging);   // (none before the first step)
      if ((s = copies_and_gather<T>(c, L, (T*)w.sHc[j], pa.out ? &pa : nullptr))) return s;
    }
    c->hlog_cur = w.slog[j];
    if ((s = substep<T>(c, lagging))) return s;   // Step 1 (near tiles only when lagging)
    {
      CopyList L;
      addM(c, L, w.sMh[j], true);
      if ((s = copies_and_gather<T>(c, L, (T*)w.sHh[j]))) return s;
    }
    void* eo[3] = {arr3<T>(w.sE[j], c, 0), arr3<T>(w.sE[j], c, 1), arr3<T>(w.sE[j], c, 2)};
    if ((s = e_step<T>(c, eo))) return s;
    for (int a = 0; a < 3; ++a) c->E[a] = eo[a];
    c->hlog_cur = w.slog[j] + lsub;
    const bool lag = lag_ok && !end;
    if ((s = substep<T>(c, lag, true))) return s;   // Step 3 (near tiles only when lagging on)
    if (lag && (s = h_far<T>(c, true))) return s;
    if (end) {
      hipLaunchKernelGGL((mmk::plane_store<T>), dim3((NY * NZ + 255) / 256), dim3(256), 0, c->stream,
                         plane_args(j, false));
      HIPCHECK(c, hipGetLastError());
    }
    lagging = lag;
    c->step++;
  }
  for (int a = 0; a < 3; ++a) c->E[a] = live.E[a];
  c->hlog_cur = nullptr;
  c->adj_recompute = false;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  std::vector<int> iters(2 * len, 1);
  if (c->nmag > 0)
    HIPCHECK(c, hipMemcpy(iters.data(), c->d_iters + 2 * m0, 2 * len * sizeof(int), hipMemcpyDeviceToHost));
  int ew = 0;
  HIPCHECK(c, hipMemcpy(&ew, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (ew & 8) return fail(c, MM_ESTATE, "a sub-step needed more iterations than the adjoint log holds (%d)", w.cap);
  for (int j = len - 1; j >= 0; --j) {
    // H^n of step j into scratch j % 2 (valid at the list entries); H^{n+1}
    // is the other scratch, filled for step j + 1, or the live fields after
    // the span's last step
    T* E1[3];
    T* H1[3];
    T* Hh[3];
    T* Hn[3];
    T* En[3];
    for (int a = 0; a < 3; ++a) {
      En[a] = j > 0 ? arr3<T>(w.sE[j - 1], c, a) : (T*)live.E[a];
      E1[a] = arr3<T>(w.sE[j], c, a);
      H1[a] = j + 1 < len ? arr3<T>(w.Hsc[(j + 1) & 1], c, a) : (T*)c->H[a];
      Hh[a] = arr3<T>(w.Hsc[2], c, a);
      Hn[a] = arr3<T>(w.Hsc[j & 1], c, a);
    }
    {
      // the compact H levels into their scratch arrays, and the flux seed at n+1
      const int bx = std::max((w.nt + 255) / 256, (NY * NZ + 255) / 256);
      hipLaunchKernelGGL((mmk::adj_step_open<T>), dim3(bx, 3), dim3(256), 0, c->stream, g, w.tidx, w.tfam, w.nt,
                         (const T*)w.sHc[j], Hn[0], Hn[1], Hn[2], (const T*)w.sHh[j], Hh[0], Hh[1], Hh[2],
                         (T*)w.Eb[1], (T*)w.Eb[2], (T*)w.Hb[1], (T*)w.Hb[2], (const T*)E1[1], (const T*)E1[2],
                         (const T*)w.sP[j], i0, c->dt * c->dy * c->dz, NY, NZ);
      HIPCHECK(c, hipGetLastError());
    }
    // Step 3: input (H, M)^{n+1/2}, output H^{n+1}
    if ((s = adj_substep<T>(c, Hh, w.sMh[j], H1, w.slog[j] + lsub, iters[2 * j + 1], true))) return s;
    // Step 2
    c->step = m0 + j;
    if ((s = adj_estep<T>(c, En, E1))) return s;
    // Step 1: input (H, M)^n, output H^{n+1/2}
    if ((s = adj_substep<T>(c, Hn, w.sM[j], Hh, w.slog[j], iters[2 * j]))) return s;
  }
  return MM_OK;
}

template <typename T>
mm_status adjoint_run(mm_ctx* c, int i0, double* grad_eps, double* grad_Ms) {
  mm_status s = adj_alloc(c);
  if (s) return s;
  AdjWork& w = *c->adjw;
  const size_t fb = c->nelem * c->esz, fd = c->nelem * sizeof(double);
  const size_t ntot = c->h_idx.size();
  const long N = c->step;
  const int sub0 = c->substep;
  const int K = w.K;
  for (int a = 0; a < 3; ++a) {
    HIPCHECK(c, hipMemsetAsync(w.Eb[a], 0, fb, c->stream));
    HIPCHECK(c, hipMemsetAsync(w.Hb[a], 0, fb, c->stream));
    HIPCHECK(c, hipMemsetAsync(w.epsb[a], 0, fd, c->stream));
  }
  if (c->nmag > 0) {
    for (int a = 0; a < 3; ++a) HIPCHECK(c, hipMemsetAsync(w.Mb[a], 0, std::max<size_t>(ntot, 1) * 8, c->stream));
    HIPCHECK(c, hipMemsetAsync(w.msf_b, 0, (size_t)c->nmag * 8, c->stream));
    HIPCHECK(c, hipMemsetAsync(w.aoms_b, 0, (size_t)c->nmag * 8, c->stream));
  }
  s = copy_state(c, w.fin, true);
  if (s) return s;
  w.cap_p = -1;
  {
    int p = 0;
    for (const ProbeRec& r : c->probes) {
      if (r.d.kind == 0) continue;
      if (r.d.i == i0) {
        w.cap_p = p;
        break;
      }
      ++p;
    }
  }
  // the E slots: the edges the E update never writes (PEC walls) keep their
  // constant values, so every slot starts as a copy of the live E
  for (void* blk : w.sE) {
    CopyList L;
    add3(c, L, blk, c->E, true);
    if ((s = run_copies(c, L))) return s;
  }
  const long nseg = (N + K - 1) / K;
  const int K2 = w.K2;
  for (long sg = nseg - 1; sg >= 0; --sg) {
    const long n0 = sg * K, n1 = std::min<long>(N, n0 + K);
    const long nsp = (n1 - n0 + K2 - 1) / K2;   // spans of at most K2 steps
    // two-level: recompute the segment once, saving the state at the start
    // of every span after the first (n0 + K2, n0 + 2 K2, ...)
    if (nsp > 1) {
      s = copy_state(c, c->ckpts[sg], false);
      if (s) return s;
      c->step = n0;
      c->substep = (int)(2 * n0);
      c->adj_recompute = true;
      c->hlog_cur = nullptr;
      // nothing is stored per step here, so the spans run as the forward ran
      // them (far tiles' fused pass, fused H-M sub-step; the same bits), each
      // ending at an integer level for its inner checkpoint
      const long keep = c->ckpt_every;
      c->ckpt_every = 0;
      for (long q = 1; q < nsp && !s; ++q) {
        s = run_steps<T>(c, K2);
        if (!s) s = copy_state(c, w.ick[q - 1], true);
      }
      c->ckpt_every = keep;
      c->adj_recompute = false;
      if (s) return s;
    }
    for (long q = nsp - 1; q >= 0; --q) {
      const long m0 = n0 + q * K2, m1 = std::min<long>(n1, m0 + K2);
      if ((s = reverse_span<T>(c, i0, m0, (int)(m1 - m0), q == 0 ? c->ckpts[sg] : w.ick[q - 1]))) return s;
    }
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  // ---- parameter chains ----
  const size_t ncells = (size_t)c->nx * c->ny * c->nz;
  std::fill(grad_Ms, grad_Ms + ncells, 0.0);
  {
    // eps_r: gathered per cell on the device, a slab of planes at a time
    // (at most ~8M cells, 64 MB), straight into the host array
    const size_t plane = (size_t)c->nx * c->ny;
    const int nk = (int)std::max<size_t>(1, std::min<size_t>((size_t)c->nz, ((size_t)1 << 23) / plane));
    double* slab = (double*)dalloc(c, plane * nk * sizeof(double));
    if (!slab) return fail(c, MM_ENOMEM, "adjoint: gradient slab allocation failed");
    const Geo g = make_geo(c);
    for (int k0 = 0; k0 < c->nz; k0 += nk) {
      const int m = std::min(nk, c->nz - k0);
      const size_t cnt = plane * m;
      hipLaunchKernelGGL(mmk::adj_eps_cells, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, c->stream, g,
                         (const double*)w.epsb[0], (const double*)w.epsb[1], (const double*)w.epsb[2], k0, m,
                         slab);
      HIPCHECK(c, hipGetLastError());
      HIPCHECK(c, hipMemcpyAsync(grad_eps + plane * k0, slab, cnt * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
      HIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    dfree(c, slab);
  }
  if (!ntot) {
    s = copy_state(c, w.fin, false);
    c->step = N;
    c->substep = sub0;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return s;
  }
  std::vector<double> mb[3], msf(c->nmag), aob(c->nmag), Msf(ntot), aoms(ntot);
  for (int a = 0; a < 3; ++a) {
    mb[a].assign(ntot, 0.0);
    HIPCHECK(c, hipMemcpy(mb[a].data(), w.Mb[a], ntot * 8, hipMemcpyDeviceToHost));
  }
  if (c->nmag) {
    HIPCHECK(c, hipMemcpy(msf.data(), w.msf_b, c->nmag * 8, hipMemcpyDeviceToHost));
    HIPCHECK(c, hipMemcpy(aob.data(), w.aoms_b, c->nmag * 8, hipMemcpyDeviceToHost));
  }
  HIPCHECK(c, hipMemcpy(Msf.data(), c->d_Ms, ntot * 8, hipMemcpyDeviceToHost));
  HIPCHECK(c, hipMemcpy(aoms.data(), c->d_aoms, ntot * 8, hipMemcpyDeviceToHost));
  for (size_t t = 0; t < (size_t)c->nmag; ++t) {
    const FaceCells& fc = c->fcells[t];
    // d L / d Ms_f: through N(M) and alpha/Ms (d(alpha/Ms)/dMs = -aoms/Ms)
    double gtot = msf[t] + aob[t] * (-aoms[t] / Msf[t]);
    // initial M0_f = v Ms_f / |v|, v = mean of Ms * m0 over the face's cells
    const double nv = std::sqrt((fc.v[0] * fc.v[0] + fc.v[1] * fc.v[1]) + fc.v[2] * fc.v[2]);
    const double vh[3] = {fc.v[0] / nv, fc.v[1] / nv, fc.v[2] / nv};
    const double m0b[3] = {mb[0][t], mb[1][t], mb[2][t]};
    const double pr = (vh[0] * m0b[0] + vh[1] * m0b[1]) + vh[2] * m0b[2];
    gtot += pr;
    double vb[3];
    for (int a = 0; a < 3; ++a) vb[a] = (Msf[t] / nv) * (m0b[a] - vh[a] * pr);
    // cells with Ms = 0 keep a zero gradient (which faces are magnetic is
    // held fixed), so an interface face adds to its magnetic cell only
    if (fc.b < 0) {   // one cell (PEC wall face)
      if (c->cell_mag[fc.a]) grad_Ms[fc.a] += gtot + ((fc.ma[0] * vb[0] + fc.ma[1] * vb[1]) + fc.ma[2] * vb[2]);
    } else {
      if (c->cell_mag[fc.a])
        grad_Ms[fc.a] += 0.5 * gtot + 0.5 * ((fc.ma[0] * vb[0] + fc.ma[1] * vb[1]) + fc.ma[2] * vb[2]);
      if (c->cell_mag[fc.b])
        grad_Ms[fc.b] += 0.5 * gtot + 0.5 * ((fc.mb[0] * vb[0] + fc.mb[1] * vb[1]) + fc.mb[2] * vb[2]);
    }
  }
  s = copy_state(c, w.fin, false);
  c->step = N;
  c->substep = sub0;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return s;
}
