// dem_api.hip -- the C ABI of libdem.so (declared in include/dem.h).
//
// Host side of one system: parameter validation, carving of the caller's
// workspace into the arrays of dem_internal.h, the per-step launch sequence
// of Sec. 4.2 (Steps 1-8), and the synchronous read-back calls, which return
// everything in the caller's original particle order.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "dem_internal.h"

using namespace dem;

struct dem_system {
  dem_params p;
  int32_t n;
  int prec;
  size_t rsz;  // sizeof(Real)
  Grid grid;
  Consts c;
  PosBuf pos[2];
  VelBuf vel[2];
  int cp, cv;  // current position / velocity buffers
  int gc;      // generation holding the committed tangential history
  int gs;      // generation holding the contact list of the current positions
  void *F[3], *T[3], *Fe[3], *Te[3];
  int32_t *cell, *rank, *perm, *scell, *counts, *cell_start;
  ScanScratch scan;
  NbrBuf nbr;
  PairGen gen[2];
  PairWork work;
  DiagBuf diag;
  int32_t *err;
  hipStream_t stream;
  dem_status sticky;
  int64_t steps;
  // phase timing (dem_profile)
  bool profiling;
  std::vector<hipEvent_t> *events;  // DEM_PROFILE_CAPACITY x (DEM_NUM_PHASES + 1)
  int64_t timed;
};

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  void *take_bytes(size_t bytes) { return take<char>(bytes); }
};

dem_status check_params(const dem_params *p, int64_t n, Grid *g) {
  // contact-list offsets are int32: n * kListCap must stay below 2^31
  if (!p || n < 0 || n > (int64_t)(INT32_MAX / kListCap)) return DEM_E_INVALID;
  if (!(p->dt > 0.0) || !isfinite(p->dt) || !(p->density > 0.0) || !(p->cell_size > 0.0)) return DEM_E_INVALID;
  if (p->law < DEM_LAW_LINEAR || p->law > DEM_LAW_SIMPLE) return DEM_E_INVALID;
  if (!(p->restitution > 0.0 && p->restitution <= 1.0) || !(p->mu >= 0.0)) return DEM_E_INVALID;
  if (p->precision != DEM_PREC_FP64 && p->precision != DEM_PREC_MIXED) return DEM_E_INVALID;
  if (p->contacts_per_particle < 1 || p->contacts_per_particle > kListCap) return DEM_E_INVALID;
  if (p->wall_mask > 0x3F) return DEM_E_INVALID;
  if (!isfinite(p->kn) || !isfinite(p->kt) || !isfinite(p->eta_t_ratio)) return DEM_E_INVALID;
  if ((int64_t)p->contacts_per_particle * n >= (int64_t)INT32_MAX) return DEM_E_INVALID;
  int64_t ncell = 1;
  for (int a = 0; a < 3; a++) {
    const double L = p->box_hi[a] - p->box_lo[a];
    if (!(L > 0.0) || !isfinite(L)) return DEM_E_INVALID;
    const double nf = floor(L / p->cell_size);
    if (nf < 1.0 || nf > 1.0e6) return DEM_E_INVALID;
    g->nc[a] = (int32_t)nf;
    g->sc[a] = (double)g->nc[a] / L;
    g->lo[a] = p->box_lo[a];
    g->hi[a] = p->box_hi[a];
    ncell *= g->nc[a];
  }
  if (ncell >= (int64_t)INT32_MAX - 1) return DEM_E_INVALID;
  g->ncell = ncell;
  return DEM_OK;
}

// Margin of the FP32 detection prefilter.  Coordinates relative to the box
// corner lie in (-w, L + w) for cells of width w, so each is rounded to FP32
// with an error of at most half an ulp of U = max(L + 2w); a difference of two
// of them is off by at most one ulp(U) plus an ulp of the cell, the norm by
// sqrt(3) times that, and the FP32 squares add a relative 2.4e-7 of the
// contact distance (<= cell).  4 ulp(U) + 1e-6 cell covers all of it, so the
// prefilter never rejects a pair that the exact FP64 test accepts.
float prefilter_eps(const Grid &g, double cell) {
  double U = 0.0;
  for (int a = 0; a < 3; a++) {
    const double L = g.hi[a] - g.lo[a];
    U = std::max(U, L + 2.0 * L / g.nc[a]);
  }
  const double ulp = ldexp(1.0, ilogb(U) - 23);
  return (float)(4.0 * ulp + 1.0e-6 * cell);
}

// Lay the arrays out in the workspace; with base == nullptr only sizes.
size_t carve(dem_system *s, char *base) {
  Carver cv{base};
  const size_t N = (size_t)(s->n > 0 ? s->n : 1);
  const size_t R = s->rsz;
  const size_t P = (size_t)s->work.Pcap;
  for (int b = 0; b < 2; b++) {
    s->pos[b].x = cv.take<double>(N);
    s->pos[b].y = cv.take<double>(N);
    s->pos[b].z = cv.take<double>(N);
    s->pos[b].r = cv.take<float>(N);
    s->pos[b].id = cv.take<int32_t>(N);
    for (int k = 0; k < 3; k++) s->vel[b].v[k] = cv.take_bytes(R * N);
    for (int k = 0; k < 3; k++) s->vel[b].w[k] = cv.take_bytes(R * N);
  }
  for (int k = 0; k < 3; k++) s->F[k] = cv.take_bytes(R * N);
  for (int k = 0; k < 3; k++) s->T[k] = cv.take_bytes(R * N);
  for (int k = 0; k < 3; k++) s->Fe[k] = cv.take_bytes(R * N);
  for (int k = 0; k < 3; k++) s->Te[k] = cv.take_bytes(R * N);
  s->cell = cv.take<int32_t>(N);
  s->rank = cv.take<int32_t>(N);
  s->perm = cv.take<int32_t>(N);
  s->scell = cv.take<int32_t>(N);
  s->counts = cv.take<int32_t>((size_t)s->grid.ncell);
  s->cell_start = cv.take<int32_t>((size_t)s->grid.ncell + 1);
  int64_t lens[4] = {0, 0, 0, 0};
  int nl = 0;
  scan_scratch_len(std::max<int64_t>(s->grid.ncell, (int64_t)N), lens, &nl);
  s->scan.nlevels = nl;
  for (int l = 0; l < 4; l++) {
    s->scan.len[l] = lens[l];
    s->scan.level[l] = l < nl ? cv.take<int32_t>((size_t)lens[l] + 1) : nullptr;
  }
  s->nbr.xyzr = cv.take<float4>(N);
  s->nbr.cnt = cv.take<int32_t>(N);
  s->nbr.nb = cv.take<int32_t>((size_t)kListCap * N);
  for (int b = 0; b < 2; b++) {
    s->gen[b].ofs = cv.take<int32_t>(N + 1);
    s->gen[b].s = cv.take<int32_t>(P);
    s->gen[b].t = cv.take<int32_t>(P);
    s->gen[b].key = cv.take<int32_t>(P);
    s->gen[b].dt = cv.take_bytes(4 * R * P);
  }
  s->work.pf = cv.take_bytes(8 * R * P);
  s->work.brank = cv.take<int32_t>(P);
  s->work.pe = cv.take<double>(P);
  s->work.pd = cv.take<double>(P);
  s->work.bcnt = cv.take<int32_t>(N);
  s->work.bofs = cv.take<int32_t>(N + 1);
  s->work.bwd = cv.take<int32_t>(P);
  s->diag.e_el = cv.take<double>(N);
  s->diag.npair = cv.take<int32_t>(N);
  s->diag.nwall = cv.take<int32_t>(N);
  s->diag.dmax = cv.take<double>(N);
  s->diag.partial = cv.take<double>((size_t)diag_blocks(s->n) * 10);
  s->diag.out = cv.take<double>(10);
  s->err = cv.take<int32_t>(64);
  return (cv.off + 255) & ~size_t(255);
}

void init_sizes(dem_system *s, const dem_params *p, int64_t n) {
  s->n = (int32_t)n;
  s->prec = p->precision;
  s->rsz = p->precision == DEM_PREC_FP64 ? sizeof(double) : sizeof(float);
  s->work.Pcap = std::max<int64_t>((int64_t)p->contacts_per_particle * n, 256);
}

void fill_consts(dem_system *s) {
  const dem_params &p = s->p;
  Consts &c = s->c;
  c.dt = p.dt;
  c.half_dt = 0.5 * p.dt;
  c.mass_c = p.density * (4.0 / 3.0) * kPi;
  const double le = log(p.restitution);
  c.alpha = p.restitution >= 1.0 ? 0.0 : -2.0 * le / sqrt(kPi * kPi + le * le);
  c.eta_t_ratio = p.eta_t_ratio;
  c.kn = p.kn;
  c.kt = p.kt;
  c.mu = p.mu;
  c.k_sp = p.simple_k[0];
  c.k_da = p.simple_k[1];
  c.k_sh = p.simple_k[2];
  for (int k = 0; k < 3; k++) c.g[k] = p.gravity[k];
  c.wall_mask = p.wall_mask;
  c.law = p.law;
}

dem_status map_err(int32_t bits) {
  if (bits & ERR_DOMAIN) return DEM_E_OUT_OF_DOMAIN;
  if (bits & ERR_NONFINITE) return DEM_E_NONFINITE;
  if (bits & ERR_OVERFLOW) return DEM_E_CONTACT_OVERFLOW;
  return DEM_OK;
}

#define HIP_TRY(expr)           \
  do {                          \
    if ((expr) != hipSuccess) { \
      (void)hipGetLastError();  \
      return DEM_E_HIP;         \
    }                           \
  } while (0)

dem_status sync_and_check(dem_system *s) {
  if (s->sticky != DEM_OK) {
    (void)hipStreamSynchronize(s->stream);
    return s->sticky;
  }
  int32_t bits = 0;
  if (hipMemcpyAsync(&bits, s->err, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess) {
    (void)hipGetLastError();
    s->sticky = DEM_E_HIP;
    return s->sticky;
  }
  s->sticky = map_err(bits);
  return s->sticky;
}

// Steps 5-6 on the current positions, into generation `g`
hipError_t build_contacts(dem_system *s, int g) {
  s->gs = g;
  return launch_contacts(s->pos[s->cp], s->nbr, s->gen[g], s->work, s->scell, s->cell_start, s->grid,
                         s->c.wall_mask, s->n, s->scan, s->err, s->stream);
}

// Steps 7-8 on the contact list of generation gs, with the committed history
// of generation gc
PairArgs pair_args(dem_system *s, int mode, void *const F[3], void *const T[3]) {
  PairArgs a;
  memset(&a, 0, sizeof(a));
  a.pos = s->pos[s->cp];
  a.vel_in = s->vel[s->cv];
  a.vel_out = s->vel[s->cv ^ 1];
  a.cur = s->gen[s->gs];
  a.old = s->gen[s->gc];
  a.w = s->work;
  a.perm = s->perm;
  a.cell = s->cell;
  for (int k = 0; k < 3; k++) {
    a.F[k] = F[k];
    a.T[k] = T[k];
  }
  a.diag = s->diag;
  a.n = s->n;
  a.mode = mode;
  a.grid = s->grid;
  a.c = s->c;
  a.err = s->err;
  return a;
}

// device -> host copy of a Real array as doubles
dem_status d2h_real(dem_system *s, const void *src, std::vector<double> &out, size_t count) {
  out.resize(count);
  if (count == 0) return DEM_OK;
  if (s->prec == DEM_PREC_FP64) {
    HIP_TRY(hipMemcpyAsync(out.data(), src, sizeof(double) * count, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else {
    std::vector<float> tmp(count);
    HIP_TRY(hipMemcpyAsync(tmp.data(), src, sizeof(float) * count, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < count; i++) out[i] = (double)tmp[i];
  }
  return DEM_OK;
}

template <typename T>
dem_status d2h(dem_system *s, const T *src, std::vector<T> &out, size_t count) {
  out.resize(count);
  if (count == 0) return DEM_OK;
  HIP_TRY(hipMemcpyAsync(out.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return DEM_OK;
}

dem_status h2d_real(dem_system *s, void *dst, const std::vector<double> &src) {
  if (src.empty()) return DEM_OK;
  if (s->prec == DEM_PREC_FP64) {
    HIP_TRY(hipMemcpyAsync(dst, src.data(), sizeof(double) * src.size(), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else {
    std::vector<float> tmp(src.size());
    for (size_t i = 0; i < src.size(); i++) tmp[i] = (float)src[i];
    HIP_TRY(hipMemcpyAsync(dst, tmp.data(), sizeof(float) * tmp.size(), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return DEM_OK;
}

template <typename T>
dem_status h2d(dem_system *s, T *dst, const std::vector<T> &src) {
  if (src.empty()) return DEM_OK;
  HIP_TRY(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return DEM_OK;
}

// per-particle vector (n x 3, original order) -> one component in slot order
void gather3(const double *src, const std::vector<int32_t> &id_at_slot, int k, std::vector<double> &out) {
  out.resize(id_at_slot.size());
  for (size_t s = 0; s < id_at_slot.size(); s++) out[s] = src[3 * (size_t)id_at_slot[s] + k];
}

struct Entry {
  int64_t a, b;
  double d[3];
};

// The contacts of a generation as sorted (a, b) keys: (lower id, higher id)
// for pairs, (id, -1 - w) for walls; with_d also reads delta_t.
dem_status read_gen(dem_system *s, const PairGen &g, bool with_d, std::vector<Entry> &out) {
  out.clear();
  if (s->n == 0) return DEM_OK;
  const size_t N = (size_t)s->n;
  std::vector<int32_t> ofs, key, id;
  dem_status st;
  if ((st = d2h(s, (const int32_t *)g.ofs, ofs, N + 1)) != DEM_OK) return st;
  const size_t P = (size_t)std::min<int64_t>(ofs[N], s->work.Pcap);
  if ((st = d2h(s, (const int32_t *)g.key, key, P)) != DEM_OK) return st;
  if ((st = d2h(s, (const int32_t *)s->pos[s->cp].id, id, N)) != DEM_OK) return st;
  std::vector<double> d;
  if (with_d && (st = d2h_real(s, g.dt, d, 4 * P)) != DEM_OK) return st;
  out.reserve(P);
  for (size_t slot = 0; slot < N; slot++) {
    for (size_t q = (size_t)ofs[slot]; q < std::min<size_t>((size_t)ofs[slot + 1], P); q++) {
      Entry e;
      const int64_t me = id[slot], other = key[q];
      e.a = other >= 0 ? std::min(me, other) : me;
      e.b = other >= 0 ? std::max(me, other) : other;
      for (int c = 0; c < 3; c++) e.d[c] = with_d ? d[4 * q + c] : 0.0;
      out.push_back(e);
    }
  }
  std::sort(out.begin(), out.end(), [](const Entry &x, const Entry &y) {
    return x.a != y.a ? x.a < y.a : x.b < y.b;
  });
  return DEM_OK;
}

dem_status fill_i32(dem_system *s, int32_t *p, size_t count, int32_t value) {
  if (count == 0) return DEM_OK;
  std::vector<int32_t> tmp(count, value);
  return h2d(s, p, tmp);
}

static void free_events(dem_system *s) {
  if (!s->events) return;
  for (hipEvent_t e : *s->events) (void)hipEventDestroy(e);
  delete s->events;
  s->events = nullptr;
}

}  // namespace

extern "C" {

const char *dem_status_string(dem_status st) {
  switch (st) {
    case DEM_OK: return "ok";
    case DEM_E_INVALID: return "invalid argument";
    case DEM_E_WORKSPACE: return "workspace missing or too small";
    case DEM_E_CONTACT_OVERFLOW: return "contact history table overflow";
    case DEM_E_OUT_OF_DOMAIN: return "particle out of domain";
    case DEM_E_NONFINITE: return "non-finite state or force";
    case DEM_E_HIP: return "HIP runtime error";
    case DEM_E_STATE: return "system handle unusable";
    case DEM_E_CAPACITY: return "output capacity too small";
  }
  return "unknown status";
}

dem_status dem_workspace_bytes(const dem_params *p, int64_t n, size_t *bytes) {
  if (!bytes) return DEM_E_INVALID;
  dem_system s;
  memset(&s, 0, sizeof(s));
  dem_status st = check_params(p, n, &s.grid);
  if (st != DEM_OK) return st;
  init_sizes(&s, p, n);
  *bytes = carve(&s, nullptr);
  return DEM_OK;
}

dem_status dem_create(const dem_params *p, int64_t n, const double *x, const double *v, const double *omega,
                      const double *r, const double *F0, const double *T0, int64_t n_hist,
                      const int64_t *hist_pairs, const double *hist_dt, void *workspace, size_t ws_bytes,
                      void *hip_stream, dem_system **out) {
  if (!out) return DEM_E_INVALID;
  *out = nullptr;
  Grid g;
  dem_status st = check_params(p, n, &g);
  if (st != DEM_OK) return st;
  if (n > 0 && (!x || !v || !omega || !r)) return DEM_E_INVALID;
  if ((F0 == nullptr) != (T0 == nullptr)) return DEM_E_INVALID;
  if (n_hist < 0 || (n_hist > 0 && (!hist_pairs || !hist_dt))) return DEM_E_INVALID;
  // radii (FP32), the cell width needed by the 27-cell search, finiteness
  std::vector<float> rf((size_t)n);
  double rmax = 0.0;
  for (int64_t i = 0; i < n; i++) {
    const float q = (float)r[i];
    if (!(q > 0.0f) || !isfinite(q)) return DEM_E_INVALID;
    rf[i] = q;
    rmax = std::max(rmax, (double)q);
  }
  if (p->cell_size < 2.0 * rmax) return DEM_E_INVALID;
  for (int64_t i = 0; i < 3 * n; i++)
    if (!isfinite(x[i]) || !isfinite(v[i]) || !isfinite(omega[i])) return DEM_E_NONFINITE;
  if (F0)
    for (int64_t i = 0; i < 3 * n; i++)
      if (!isfinite(F0[i]) || !isfinite(T0[i])) return DEM_E_NONFINITE;
  const bool keep_hist = p->law != DEM_LAW_SIMPLE && n_hist > 0;
  if (keep_hist) {
    for (int64_t k = 0; k < n_hist; k++) {
      const int64_t a = hist_pairs[2 * k], b = hist_pairs[2 * k + 1];
      const bool ok = a >= 0 && a < n && ((b > a && b < n) || (b < 0 && b >= -6));
      if (!ok) return DEM_E_INVALID;
      for (int q = 0; q < 3; q++)
        if (!isfinite(hist_dt[3 * k + q])) return DEM_E_NONFINITE;
    }
  }

  dem_system *s = new (std::nothrow) dem_system;
  if (!s) return DEM_E_INVALID;
  memset((void *)s, 0, sizeof(*s));
  s->p = *p;
  init_sizes(s, p, n);
  s->grid = g;
  s->stream = (hipStream_t)hip_stream;
  s->nbr.eps = prefilter_eps(g, p->cell_size);
  fill_consts(s);
  const size_t need = carve(s, nullptr);
  if (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255)) {
    delete s;
    return DEM_E_WORKSPACE;
  }
  carve(s, (char *)workspace);

  auto fail = [&](dem_status e) {
    (void)hipStreamSynchronize(s->stream);
    free_events(s);
    delete s;
    return e;
  };
  const size_t N = (size_t)n;
  if (fill_i32(s, s->err, 64, 0) != DEM_OK) return fail(DEM_E_HIP);
  // upload in original order into buffer 0
  std::vector<int32_t> ids(N);
  std::iota(ids.begin(), ids.end(), 0);
  {
    std::vector<double> tmp;
    const PosBuf &pb = s->pos[0];
    double *dst[3] = {pb.x, pb.y, pb.z};
    for (int k = 0; k < 3; k++) {
      gather3(x, ids, k, tmp);
      if (h2d(s, dst[k], tmp) != DEM_OK) return fail(DEM_E_HIP);
    }
    for (int k = 0; k < 3; k++) {
      gather3(v, ids, k, tmp);
      if (h2d_real(s, s->vel[0].v[k], tmp) != DEM_OK) return fail(DEM_E_HIP);
      gather3(omega, ids, k, tmp);
      if (h2d_real(s, s->vel[0].w[k], tmp) != DEM_OK) return fail(DEM_E_HIP);
    }
    if (h2d(s, pb.r, rf) != DEM_OK || h2d(s, pb.id, ids) != DEM_OK) return fail(DEM_E_HIP);
  }
  // Steps 2-4 on the initial positions
  if (launch_hash(s->pos[0], s->n, s->grid, s->cell, s->err, s->stream) != hipSuccess) return fail(DEM_E_HIP);
  if (launch_sort(s->cell, s->pos[0].id, s->n, s->grid.ncell, s->counts, s->rank, s->cell_start, s->perm,
                  s->scan, s->stream) != hipSuccess)
    return fail(DEM_E_HIP);
  if (launch_reorder(s->prec, s->pos[0], s->vel[0], s->pos[1], s->vel[1], s->perm, s->cell, s->scell,
                     s->nbr.xyzr, s->grid, s->n, s->stream) != hipSuccess)
    return fail(DEM_E_HIP);
  s->cp = 1;
  s->cv = 1;
  s->gc = 0;
  // Steps 5-6: the contacts of the initial positions go to generation 1
  if (build_contacts(s, 1) != hipSuccess) return fail(DEM_E_HIP);
  st = sync_and_check(s);
  if (st != DEM_OK) return fail(st);
  std::vector<int32_t> id_at_slot;
  if (d2h(s, s->pos[1].id, id_at_slot, N) != DEM_OK) return fail(DEM_E_HIP);
  // the given history becomes generation 0, filed under the lower slot of
  // each pair (the particle for a wall) in the sorted order
  {
    std::vector<int32_t> slot_of(N);
    for (size_t sl = 0; sl < N; sl++) slot_of[id_at_slot[sl]] = (int32_t)sl;
    std::vector<int32_t> cnt(N + 1, 0);
    struct Rec {
      int32_t owner, key;
      double d[3];
    };
    std::vector<Rec> recs;
    if (keep_hist) {
      recs.reserve((size_t)n_hist);
      for (int64_t k = 0; k < n_hist; k++) {
        const int64_t a = hist_pairs[2 * k], b = hist_pairs[2 * k + 1];
        Rec rc;
        if (b >= 0) {
          const int32_t sa = slot_of[a], sb = slot_of[b];
          rc.owner = std::min(sa, sb);
          rc.key = (int32_t)(sa < sb ? b : a);
        } else {
          rc.owner = slot_of[a];
          rc.key = (int32_t)b;
        }
        memcpy(rc.d, hist_dt + 3 * k, sizeof(rc.d));
        recs.push_back(rc);
      }
      std::stable_sort(recs.begin(), recs.end(), [](const Rec &u, const Rec &w) { return u.owner < w.owner; });
      for (size_t k = 1; k < recs.size(); k++)
        if (recs[k].owner == recs[k - 1].owner && recs[k].key == recs[k - 1].key) return fail(DEM_E_INVALID);
    }
    if ((int64_t)recs.size() > s->work.Pcap) return fail(DEM_E_CONTACT_OVERFLOW);
    std::vector<int32_t> ofs(N + 1, 0), key(recs.size());
    std::vector<double> d(4 * recs.size(), 0.0);
    for (const Rec &rc : recs) ofs[rc.owner + 1]++;
    for (size_t k = 0; k < N; k++) ofs[k + 1] += ofs[k];
    for (size_t k = 0; k < recs.size(); k++) {
      key[k] = recs[k].key;
      for (int c = 0; c < 3; c++) d[4 * k + c] = recs[k].d[c];
    }
    const PairGen &g0 = s->gen[0];
    if (h2d(s, g0.ofs, ofs) != DEM_OK || h2d(s, g0.key, key) != DEM_OK || h2d_real(s, g0.dt, d) != DEM_OK)
      return fail(DEM_E_HIP);
  }
  // forces of the initial state
  if (F0) {
    std::vector<double> tmp;
    for (int k = 0; k < 3; k++) {
      gather3(F0, id_at_slot, k, tmp);
      if (h2d_real(s, s->F[k], tmp) != DEM_OK) return fail(DEM_E_HIP);
      gather3(T0, id_at_slot, k, tmp);
      if (h2d_real(s, s->T[k], tmp) != DEM_OK) return fail(DEM_E_HIP);
    }
  } else {
    PairArgs a = pair_args(s, 0, s->F, s->T);
    if (launch_forces(s->prec, a, s->stream) != hipSuccess) return fail(DEM_E_HIP);
  }
  st = sync_and_check(s);
  if (st != DEM_OK) return fail(st);
  *out = s;
  return DEM_OK;
}

dem_status dem_step(dem_system *s, int64_t nsteps) {
  if (!s) return DEM_E_STATE;
  if (nsteps < 0) return DEM_E_INVALID;
  if (s->sticky != DEM_OK) return s->sticky;
  bool drifted = false;  // the previous step's closing pass already ran Steps 1-2
  for (int64_t k = 0; k < nsteps; k++) {
    hipEvent_t *ev = nullptr;
    if (s->profiling && s->timed < DEM_PROFILE_CAPACITY) {
      ev = s->events->data() + (size_t)s->timed * (DEM_NUM_PHASES + 1);
      s->timed++;
    }
    auto mark = [&](int phase) {
      if (ev) (void)hipEventRecord(ev[phase], s->stream);
    };
    mark(0);
    // Step 1 (opening half kick, drift) fused with Step 2 (hash)
    if (!drifted && launch_kick_drift_hash(s->prec, s->pos[s->cp], s->vel[s->cv], s->F, s->T, s->n, s->c,
                                           s->grid, s->cell, s->err, s->stream) != hipSuccess)
      return s->sticky = DEM_E_HIP;
    mark(1);
    // Step 3
    if (launch_sort(s->cell, s->pos[s->cp].id, s->n, s->grid.ncell, s->counts, s->rank, s->cell_start, s->perm,
                    s->scan, s->stream) != hipSuccess)
      return s->sticky = DEM_E_HIP;
    mark(2);
    // Step 4
    if (launch_reorder(s->prec, s->pos[s->cp], s->vel[s->cv], s->pos[s->cp ^ 1], s->vel[s->cv ^ 1], s->perm,
                       s->cell, s->scell, s->nbr.xyzr, s->grid, s->n, s->stream) != hipSuccess)
      return s->sticky = DEM_E_HIP;
    s->cp ^= 1;
    s->cv ^= 1;
    mark(3);
    // Steps 5-6 into the generation that does not hold the committed history
    if (build_contacts(s, s->gc ^ 1) != hipSuccess) return s->sticky = DEM_E_HIP;
    mark(4);
    // Steps 7-8 and the closing half kick; the new history is committed.
    // Between two steps of this call the closing pass also runs the next
    // step's opening kick, drift and hash (the state stays in registers).
    drifted = k + 1 < nsteps;
    PairArgs a = pair_args(s, MODE_WRITE_HIST | MODE_KICK | MODE_OLD_PERM | (drifted ? MODE_DRIFT : 0), s->F,
                           s->T);
    if (launch_forces(s->prec, a, s->stream) != hipSuccess) return s->sticky = DEM_E_HIP;
    mark(5);
    s->cv ^= 1;
    s->gc = s->gs;
    s->steps++;
  }
  return DEM_OK;
}

dem_status dem_sync(dem_system *s) {
  if (!s) return DEM_E_STATE;
  return sync_and_check(s);
}

dem_status dem_forces(dem_system *s, double *F, double *T) {
  if (!s) return DEM_E_STATE;
  if (!F || !T) return DEM_E_INVALID;
  dem_status st = sync_and_check(s);
  if (st != DEM_OK) return st;
  PairArgs a = pair_args(s, 0, s->Fe, s->Te);
  if (launch_forces(s->prec, a, s->stream) != hipSuccess) return s->sticky = DEM_E_HIP;
  if ((st = sync_and_check(s)) != DEM_OK) return st;
  const size_t N = (size_t)s->n;
  std::vector<int32_t> id;
  if ((st = d2h(s, s->pos[s->cp].id, id, N)) != DEM_OK) return st;
  std::vector<double> tmp;
  for (int k = 0; k < 3; k++) {
    if ((st = d2h_real(s, s->Fe[k], tmp, N)) != DEM_OK) return st;
    for (size_t i = 0; i < N; i++) F[3 * (size_t)id[i] + k] = tmp[i];
    if ((st = d2h_real(s, s->Te[k], tmp, N)) != DEM_OK) return st;
    for (size_t i = 0; i < N; i++) T[3 * (size_t)id[i] + k] = tmp[i];
  }
  return DEM_OK;
}

dem_status dem_read_state(dem_system *s, double *x, double *v, double *omega, double *F, double *T) {
  if (!s) return DEM_E_STATE;
  dem_status st = sync_and_check(s);
  if (st != DEM_OK) return st;
  const size_t N = (size_t)s->n;
  std::vector<int32_t> id;
  if ((st = d2h(s, s->pos[s->cp].id, id, N)) != DEM_OK) return st;
  if (x) {
    std::vector<double> tmp;
    const double *src[3] = {s->pos[s->cp].x, s->pos[s->cp].y, s->pos[s->cp].z};
    for (int k = 0; k < 3; k++) {
      if ((st = d2h(s, src[k], tmp, N)) != DEM_OK) return st;
      for (size_t i = 0; i < N; i++) x[3 * (size_t)id[i] + k] = tmp[i];
    }
  }
  void *const *arrs[4] = {s->vel[s->cv].v, s->vel[s->cv].w, s->F, s->T};
  double *outs[4] = {v, omega, F, T};
  for (int q = 0; q < 4; q++) {
    if (!outs[q]) continue;
    std::vector<double> tmp;
    for (int k = 0; k < 3; k++) {
      if ((st = d2h_real(s, arrs[q][k], tmp, N)) != DEM_OK) return st;
      for (size_t i = 0; i < N; i++) outs[q][3 * (size_t)id[i] + k] = tmp[i];
    }
  }
  return DEM_OK;
}

dem_status dem_read_contacts(dem_system *s, int64_t cap, int64_t *n_out, int64_t *pairs, double *delta_t) {
  if (!s) return DEM_E_STATE;
  if (!n_out) return DEM_E_INVALID;
  dem_status st = sync_and_check(s);
  if (st != DEM_OK) return st;
  std::vector<Entry> e;
  if (s->p.law != DEM_LAW_SIMPLE && (st = read_gen(s, s->gen[s->gc], true, e)) != DEM_OK) return st;
  *n_out = (int64_t)e.size();
  if ((int64_t)e.size() > cap) return DEM_E_CAPACITY;
  for (size_t k = 0; k < e.size(); k++) {
    if (pairs) {
      pairs[2 * k] = e[k].a;
      pairs[2 * k + 1] = e[k].b;
    }
    if (delta_t)
      for (int q = 0; q < 3; q++) delta_t[3 * k + q] = e[k].d[q];
  }
  return DEM_OK;
}

dem_status dem_contacts(dem_system *s, int64_t cap, int64_t *n_out, int64_t *pairs) {
  if (!s) return DEM_E_STATE;
  if (!n_out) return DEM_E_INVALID;
  dem_status st = sync_and_check(s);
  if (st != DEM_OK) return st;
  std::vector<Entry> e;
  if ((st = read_gen(s, s->gen[s->gs], false, e)) != DEM_OK) return st;
  *n_out = (int64_t)e.size();
  if ((int64_t)e.size() > cap) return DEM_E_CAPACITY;
  for (size_t k = 0; k < e.size() && pairs; k++) {
    pairs[2 * k] = e[k].a;
    pairs[2 * k + 1] = e[k].b;
  }
  return DEM_OK;
}

dem_status dem_read_grid(dem_system *s, int32_t *cell_of_id, int32_t *id_at_slot, int32_t *cell_start) {
  if (!s) return DEM_E_STATE;
  dem_status st = sync_and_check(s);
  if (st != DEM_OK) return st;
  const size_t N = (size_t)s->n;
  std::vector<int32_t> id, sc;
  if ((st = d2h(s, s->pos[s->cp].id, id, N)) != DEM_OK) return st;
  if (cell_of_id) {
    if ((st = d2h(s, (const int32_t *)s->scell, sc, N)) != DEM_OK) return st;
    for (size_t i = 0; i < N; i++) cell_of_id[id[i]] = sc[i];
  }
  if (id_at_slot && N) memcpy(id_at_slot, id.data(), 4 * N);
  if (cell_start) {
    std::vector<int32_t> cs;
    if ((st = d2h(s, (const int32_t *)s->cell_start, cs, (size_t)s->grid.ncell + 1)) != DEM_OK) return st;
    memcpy(cell_start, cs.data(), 4 * cs.size());
  }
  return DEM_OK;
}

dem_status dem_grid_dims(dem_system *s, int32_t dims[3]) {
  if (!s) return DEM_E_STATE;
  if (!dims) return DEM_E_INVALID;
  for (int a = 0; a < 3; a++) dims[a] = s->grid.nc[a];
  return DEM_OK;
}

dem_status dem_diagnostics(dem_system *s, double out[10]) {
  if (!s) return DEM_E_STATE;
  if (!out) return DEM_E_INVALID;
  dem_status st = sync_and_check(s);
  if (st != DEM_OK) return st;
  PairArgs a = pair_args(s, MODE_DIAG, s->Fe, s->Te);
  if (launch_forces(s->prec, a, s->stream) != hipSuccess) return s->sticky = DEM_E_HIP;
  if (launch_diag_reduce(s->prec, s->pos[s->cp], s->vel[s->cv], s->diag, s->n, s->c, s->grid, s->stream) !=
      hipSuccess)
    return s->sticky = DEM_E_HIP;
  if ((st = sync_and_check(s)) != DEM_OK) return st;
  std::vector<double> o;
  if ((st = d2h(s, (const double *)s->diag.out, o, 10)) != DEM_OK) return st;
  memcpy(out, o.data(), 10 * sizeof(double));
  return DEM_OK;
}

dem_status dem_set_radii(dem_system *s, const double *r) {
  if (!s) return DEM_E_STATE;
  if (s->n > 0 && !r) return DEM_E_INVALID;
  dem_status st = sync_and_check(s);
  if (st != DEM_OK) return st;
  const size_t N = (size_t)s->n;
  std::vector<float> rf(N);
  double rmax = 0.0;
  for (size_t i = 0; i < N; i++) {
    const float q = (float)r[i];
    if (!(q > 0.0f) || !isfinite(q)) return DEM_E_INVALID;
    rf[i] = q;
    rmax = std::max(rmax, (double)q);
  }
  if (s->p.cell_size < 2.0 * rmax) return DEM_E_INVALID;
  std::vector<int32_t> id;
  if ((st = d2h(s, s->pos[s->cp].id, id, N)) != DEM_OK) return st;
  std::vector<float> slot_r(N);
  for (size_t k = 0; k < N; k++) slot_r[k] = rf[id[k]];
  if (N) {
    if ((st = h2d(s, s->pos[s->cp].r, slot_r)) != DEM_OK) return st;
    HIP_TRY(launch_xyzr(s->pos[s->cp], s->nbr.xyzr, s->grid, s->n, s->stream));
    // the contact list of the new radii, beside the committed history
    HIP_TRY(build_contacts(s, s->gc ^ 1));
  }
  return sync_and_check(s);
}

dem_status dem_profile(dem_system *s, int enable) {
  if (!s) return DEM_E_STATE;
  if (enable && !s->events) {
    const size_t cnt = (size_t)DEM_PROFILE_CAPACITY * (DEM_NUM_PHASES + 1);
    s->events = new (std::nothrow) std::vector<hipEvent_t>(cnt, nullptr);
    if (!s->events) return DEM_E_INVALID;
    for (size_t k = 0; k < cnt; k++)
      if (hipEventCreate(&(*s->events)[k]) != hipSuccess) {
        (void)hipGetLastError();
        free_events(s);
        return DEM_E_HIP;
      }
  }
  s->profiling = enable != 0;
  s->timed = 0;
  return DEM_OK;
}

dem_status dem_profile_read(dem_system *s, double ms[DEM_NUM_PHASES], int64_t *steps) {
  if (!s) return DEM_E_STATE;
  if (!ms || !steps) return DEM_E_INVALID;
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int p = 0; p < DEM_NUM_PHASES; p++) ms[p] = 0.0;
  for (int64_t k = 0; k < s->timed; k++) {
    hipEvent_t *ev = s->events->data() + (size_t)k * (DEM_NUM_PHASES + 1);
    for (int p = 0; p < DEM_NUM_PHASES; p++) {
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, ev[p], ev[p + 1]));
      ms[p] += (double)t;
    }
  }
  *steps = s->timed;
  s->timed = 0;
  return DEM_OK;
}

dem_status dem_destroy(dem_system *s) {
  if (!s) return DEM_E_STATE;
  (void)hipStreamSynchronize(s->stream);
  free_events(s);
  delete s;
  return DEM_OK;
}

}  // extern "C"
