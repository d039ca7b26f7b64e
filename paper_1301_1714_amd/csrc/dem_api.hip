// dem_api.hip -- the C ABI of libdem.so (declared in include/dem.h).
//
// Host side of an engine of S independent systems (one for dem_system, many
// for dem_batch): parameter validation, carving of the caller's workspace
// into the arrays of dem_internal.h, the per-step launch sequence of
// Sec. 4.2 (Steps 1-8), optional replay of a step from HIP graphs, and the
// synchronous read-back calls, which return everything in the caller's
// original particle order.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "dem_internal.h"

using namespace dem;

namespace {

constexpr double kPi = 3.14159265358979323846;


struct Engine {
  int32_t S = 0;
  int32_t n = 0;  // particles of all systems
  int prec = 0;
  int law = 0;
  size_t rsz = 0;  // sizeof(Real)
  std::vector<dem_params> params;
  std::vector<SysInfo> info;  // host copy of the system table
  std::vector<int32_t> bsys_h, bfirst_h;
  std::vector<int32_t> psys_h;  // system of each slot
  std::vector<int4> tiles_h;  // detection work items
  std::vector<int4> runs_h;   // wave detection work items
  int64_t ncell = 0;  // cells of all systems
  int32_t K = 1;      // owned contacts per particle at most (largest contacts_per_particle)
  bool has_mt = false;  // some system may have a material-pair table
  bool has_terms = false;  // some system has optional contact terms
  int64_t nmat = 0;     // entries of all systems' tables (max_materials^2 each)
  // device
  SysInfo *tab = nullptr;
  PairK *mat = nullptr;
  int32_t *psys = nullptr, *bsys = nullptr, *bfirst = nullptr;
  int4 *tiles = nullptr;
  int4 *runs = nullptr;
  StepCtl ctl{};
  std::vector<int32_t> left_h;  // source of the ctl.left upload
  hipEvent_t left_ev = nullptr;  // that upload has been read
  bool left_pending = false;
  PosBuf pos[2];
  VelBuf vel[2];
  int cp = 0, cv = 0;  // current position / velocity buffers
  int gc = 0;          // generation holding the committed tangential history
  void *F[3], *T[3], *Fe[3], *Te[3];
  int32_t *cell = nullptr, *rank = nullptr, *perm = nullptr, *scell = nullptr, *counts = nullptr,
          *cell_start = nullptr;
  uint8_t *reflag = nullptr;  // [ncell, padded to whole words] cells the next sort must order again
  ScanScratch scan{};
  NbrBuf nbr{};
  HistGen hist[2];
  PairWork work{};
  DiagBuf diag{};
  int32_t *err = nullptr;
  unsigned long long *vmax = nullptr;  // [S] largest speeds (dem_max_speed)
  hipStream_t stream = nullptr;
  dem_status sticky = DEM_OK;
  // phase timing
  bool profiling = false;
  std::vector<hipEvent_t> events;  // DEM_PROFILE_CAPACITY x (DEM_NUM_PHASES + 1)
  int64_t timed = 0;
  // graph replay of Steps 3-8, one graph per history generation
  bool use_graph = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int gexec_cp[2] = {-1, -1};  // the position buffer each graph was captured with
  int32_t ndirect = 0;         // systems swept by the direct detection kernel (reach 1)
  int32_t ndirect2 = 0;        // the same with reach 2

  Layout layout() const {
    Layout L;
    L.tab = tab;
    L.mat = mat;
    L.psys = psys;
    L.bsys = bsys;
    L.bfirst = bfirst;
    L.tiles = tiles;
    L.runs = runs;
    L.nblocks = (int32_t)bsys_h.size();
    L.ntiles = (int32_t)tiles_h.size();
    L.nruns = (int32_t)runs_h.size();
    L.ndirect = ndirect;
    L.ndirect2 = ndirect2;
    L.n = n;
    L.S = S;
    return L;
  }
};

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
  if (!p || n < 0 || n > kMaxParticles) return DEM_E_INVALID;
  if (!(p->dt > 0.0) || !isfinite(p->dt) || !(p->density > 0.0) || !(p->cell_size > 0.0)) return DEM_E_INVALID;
  if (p->law < DEM_LAW_LINEAR || p->law > DEM_LAW_SIMPLE) return DEM_E_INVALID;
  if (!(p->restitution > 0.0 && p->restitution <= 1.0) || !(p->mu >= 0.0)) return DEM_E_INVALID;
  if (p->precision != DEM_PREC_FP64 && p->precision != DEM_PREC_MIXED) return DEM_E_INVALID;
  if (p->contacts_per_particle < 1 || p->contacts_per_particle > kListCap) return DEM_E_INVALID;
  if (p->wall_mask > 0x3F) return DEM_E_INVALID;
  if (!isfinite(p->kn) || !isfinite(p->kt) || !isfinite(p->eta_t_ratio)) return DEM_E_INVALID;
  if (p->tile_cells < -1 || p->tile_cells > kMaxTile) return DEM_E_INVALID;
  if (p->cell_divisor < 1 || p->cell_divisor > kMaxReach) return DEM_E_INVALID;
  if (p->cell_divisor > 1 && p->tile_cells != 0) return DEM_E_INVALID;  // the other shapes sweep 27 cells
  if (p->max_materials < 0 || p->max_materials > kMaxMaterials) return DEM_E_INVALID;
  if (p->nplates < 0 || p->nplates > kMaxPlates) return DEM_E_INVALID;
  for (int k = 0; k < p->nplates; k++) {
    const dem_plate &q = p->plates[k];
    if (q.axis < 0 || q.axis > 2 || !isfinite(q.at) || !isfinite(q.lo[0]) || !isfinite(q.lo[1]) ||
        !isfinite(q.hi[0]) || !isfinite(q.hi[1]) || !(q.lo[0] <= q.hi[0]) || !(q.lo[1] <= q.hi[1]))
      return DEM_E_INVALID;
  }
  if ((p->terms & ~(uint32_t)(DEM_TERM_COHESION | DEM_TERM_ROLLING)) != 0) return DEM_E_INVALID;
  if (p->terms != 0 && (p->law == DEM_LAW_SIMPLE || !isfinite(p->cohesion) || !(p->rolling_mu >= 0.0) ||
                        !isfinite(p->rolling_mu)))
    return DEM_E_INVALID;
  const double width = p->cell_size / p->cell_divisor;
  int64_t ncell = 1;
  for (int a = 0; a < 3; a++) {
    const double L = p->box_hi[a] - p->box_lo[a];
    if (!(L > 0.0) || !isfinite(L)) return DEM_E_INVALID;
    const double nf = floor(L / width);
    if (nf < 1.0 || nf > 1.0e6) return DEM_E_INVALID;
    g->nc[a] = (int32_t)nf;
    g->sc[a] = (double)g->nc[a] / L;
    g->lo[a] = p->box_lo[a];
    g->hi[a] = p->box_hi[a];
    ncell *= g->nc[a];
  }
  if (ncell >= (int64_t)INT32_MAX - 1) return DEM_E_INVALID;
  g->ncell = (int32_t)ncell;
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

// Eq. 10's alpha for restitution e: -2 ln e / sqrt(pi^2 + ln^2 e), which
// makes a linear contact's restitution exactly e.  One function for the
// system constants and the material tables, so that a table entry equal to
// the parameters gives the same bits (the compiler may contract the
// expression differently in two places).
double alpha_of(double e) {
  if (e >= 1.0) return 0.0;
  const double le = log(e);
  return -2.0 * le / sqrt(kPi * kPi + le * le);
}

void fill_consts(const dem_params &p, Consts &c) {
  c.dt = p.dt;
  c.half_dt = 0.5 * p.dt;
  c.mass_c = p.density * (4.0 / 3.0) * kPi;
  c.alpha = alpha_of(p.restitution);
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
  c.terms = p.terms;
  c.cohesion = (p.terms & DEM_TERM_COHESION) ? p.cohesion : 0.0;
  c.rolling_mu = (p.terms & DEM_TERM_ROLLING) ? p.rolling_mu : 0.0;
}

// Validate the systems and lay out slot, cell and block ranges (no device
// memory yet).  All systems share one precision and one contact law.
dem_status plan(Engine &e, int32_t S, const dem_params *p, const int64_t *n) {
  if (S < 1 || !p || !n) return DEM_E_INVALID;
  e.S = S;
  e.params.assign(p, p + S);
  e.info.assign(S, SysInfo{});
  e.prec = p[0].precision;
  e.law = p[0].law;
  int64_t ntot = 0, ctot = 0;
  e.K = 1;
  e.bsys_h.clear();
  e.bfirst_h.clear();
  e.tiles_h.clear();
  e.runs_h.clear();
  e.ndirect = 0;
  e.ndirect2 = 0;
  e.has_mt = false;
  e.has_terms = false;
  e.nmat = 0;
  for (int32_t k = 0; k < S; k++) {
    SysInfo &si = e.info[k];
    memset(&si, 0, sizeof(si));
    dem_status st = check_params(&p[k], n[k], &si.g);
    if (st != DEM_OK) return st;
    if (p[k].precision != e.prec || p[k].law != e.law) return DEM_E_INVALID;
    fill_consts(p[k], si.c);
    si.nplates = p[k].nplates;
    for (int q = 0; q < p[k].nplates; q++) {
      const dem_plate &d = p[k].plates[q];
      si.plates[q] = Plate{d.axis, 0, d.at, {d.lo[0], d.lo[1]}, {d.hi[0], d.hi[1]}};
    }
    si.eps = prefilter_eps(si.g, p[k].cell_size);
    si.reach = p[k].cell_divisor;
    si.kcap = p[k].contacts_per_particle;
    e.K = std::max(e.K, si.kcap);
    si.ntypes = 0;  // one material until dem_set_materials
    si.wall_type = 0;
    si.mat0 = (int32_t)e.nmat;
    e.nmat += (int64_t)p[k].max_materials * p[k].max_materials;
    e.has_mt = e.has_mt || p[k].max_materials > 0;
    e.has_terms = e.has_terms || p[k].terms != 0;
    si.p0 = (int32_t)ntot;
    si.n = (int32_t)n[k];
    si.g.c0 = (int32_t)ctot;
    // per-particle kernels: blocks of kBlock slots that never straddle systems
    for (int64_t b = 0; b < n[k]; b += kBlock) {
      e.bsys_h.push_back(k);
      e.bfirst_h.push_back((int32_t)(ntot + b));
    }
    // detection tiles: runs of T cells along x in every (y, z) row
    const int32_t T = p[k].tile_cells;
    const int32_t nx = si.g.nc[0], rows = si.g.nc[1] * si.g.nc[2];
    si.tile = T;
    if (n[k] > 0 && T == 0) (si.reach == 1 ? e.ndirect : e.ndirect2)++;
    if (n[k] > 0 && T < 0) {
      if ((int64_t)e.runs_h.size() + (int64_t)rows * ((nx + kRunCells - 1) / kRunCells) >= (int64_t)INT32_MAX)
        return DEM_E_INVALID;
      for (int32_t row = 0; row < rows; row++)
        for (int32_t x0 = 0; x0 < nx; x0 += kRunCells)
          e.runs_h.push_back(make_int4(k, row, x0, std::min(x0 + kRunCells, nx) - 1));
    }
    if (n[k] > 0 && T > 0) {
      if ((int64_t)e.tiles_h.size() + (int64_t)rows * ((nx + T - 1) / T) >= (int64_t)INT32_MAX)
        return DEM_E_INVALID;
      for (int32_t row = 0; row < rows; row++)
        for (int32_t x0 = 0; x0 < nx; x0 += T) e.tiles_h.push_back(make_int4(k, row, x0, std::min(x0 + T, nx) - 1));
    }
    ntot += n[k];
    ctot += si.g.ncell;
    if (ntot > kMaxParticles || ctot >= (int64_t)INT32_MAX - 1) return DEM_E_INVALID;
  }
  e.n = (int32_t)ntot;
  e.ncell = ctot;
  // contact indices (backward entries, history starts) are int32
  if ((int64_t)e.bsys_h.size() * kBlock * e.K >= (int64_t)INT32_MAX) return DEM_E_INVALID;
  e.rsz = e.prec == DEM_PREC_FP64 ? sizeof(double) : sizeof(float);
  e.left_h.assign(S, 0);
  return DEM_OK;
}

// Lay the arrays out in the workspace; with base == nullptr only sizes.
size_t carve(Engine &e, char *base) {
  Carver cv{base};
  const size_t N = (size_t)(e.n > 0 ? e.n : 1);
  const size_t R = e.rsz;
  const size_t P = (size_t)e.K * N;  // owned-contact lists [K][N]
  const size_t S = (size_t)e.S;
  const size_t B = std::max<size_t>(e.bsys_h.size(), 1);
  const size_t PB = B * (size_t)kBlock * (size_t)e.K;  // per-contact arrays: kBlock * K entries per block
  e.tab = cv.take<SysInfo>(S);
  e.mat = cv.take<PairK>(std::max<size_t>((size_t)e.nmat, 1));
  e.psys = cv.take<int32_t>(N);
  e.bsys = cv.take<int32_t>(B);
  e.bfirst = cv.take<int32_t>(B);
  e.tiles = cv.take<int4>(std::max<size_t>(e.tiles_h.size(), 1));
  e.runs = cv.take<int4>(std::max<size_t>(e.runs_h.size(), 1));
  e.ctl.step = cv.take<int32_t>(64);
  e.ctl.left = cv.take<int32_t>(S);
  for (int b = 0; b < 2; b++) {
    e.pos[b].x = cv.take<double>(N);
    e.pos[b].y = cv.take<double>(N);
    e.pos[b].z = cv.take<double>(N);
    e.pos[b].r = cv.take<float>(N);
    e.pos[b].id = cv.take<int32_t>(N);
    e.pos[b].mt = e.has_mt ? cv.take<int32_t>(N) : nullptr;
    for (int k = 0; k < 3; k++) e.vel[b].v[k] = cv.take_bytes(R * N);
    for (int k = 0; k < 3; k++) e.vel[b].w[k] = cv.take_bytes(R * N);
  }
  for (int k = 0; k < 3; k++) e.F[k] = cv.take_bytes(R * N);
  for (int k = 0; k < 3; k++) e.T[k] = cv.take_bytes(R * N);
  for (int k = 0; k < 3; k++) e.Fe[k] = cv.take_bytes(R * N);
  for (int k = 0; k < 3; k++) e.Te[k] = cv.take_bytes(R * N);
  e.cell = cv.take<int32_t>(N);
  e.rank = cv.take<int32_t>(N);
  e.perm = cv.take<int32_t>(N);
  e.scell = cv.take<int32_t>(N);
  e.counts = cv.take<int32_t>((size_t)e.ncell);
  e.reflag = (uint8_t *)cv.take<int32_t>(((size_t)e.ncell + 3) / 4);
  e.cell_start = cv.take<int32_t>((size_t)e.ncell + 1);
  int64_t lens[4] = {0, 0, 0, 0};
  int nl = 0;
  scan_scratch_len(e.ncell, lens, &nl);
  e.scan.nlevels = nl;
  for (int l = 0; l < 4; l++) {
    e.scan.len[l] = lens[l];
    e.scan.level[l] = l < nl ? cv.take<int32_t>((size_t)lens[l] + 1) : nullptr;
  }
  e.nbr.xyzr = cv.take<float4>(N);
  e.nbr.xq = cv.take<uint2>(N + 1);  // one pad record: detection loads records in pairs
  e.nbr.fcnt = cv.take<int32_t>(N);
  e.nbr.pst = cv.take_bytes((e.prec == DEM_PREC_FP64 ? sizeof(PState<double>) : sizeof(PState<float>)) * N);
  e.nbr.nb = cv.take<int32_t>(P);
  e.nbr.K = e.K;
  for (int b = 0; b < 2; b++) {
    e.hist[b].cnt = cv.take<int32_t>(N);
    e.hist[b].start = cv.take<int32_t>(N);
    e.hist[b].ent = cv.take_bytes(4 * R * PB);
  }
  e.work.pf = cv.take_bytes(6 * R * PB);
  e.work.pc = e.has_terms ? cv.take_bytes(4 * R * PB) : nullptr;
  e.work.pe = cv.take<double>(PB);
  e.work.pd = cv.take<double>(PB);
  e.work.qs = cv.take<int32_t>(N);
  e.work.back = cv.take<int2>((size_t)B * kBackCap);
  e.work.nback = cv.take<int32_t>(B);
  e.diag.e_el = cv.take<double>(N);
  e.diag.npair = cv.take<int32_t>(N);
  e.diag.nwall = cv.take<int32_t>(N);
  e.diag.dmax = cv.take<double>(N);
  e.diag.partial = cv.take<double>(B * 10);
  e.diag.out = cv.take<double>(S * 10);
  e.err = cv.take<int32_t>(64);
  e.vmax = cv.take<unsigned long long>(S);
  return (cv.off + 255) & ~size_t(255);
}

dem_status map_err(int32_t bits) {
  if (bits & ERR_DOMAIN) return DEM_E_OUT_OF_DOMAIN;
  if (bits & ERR_NONFINITE) return DEM_E_NONFINITE;
  if (bits & ERR_OVERFLOW) return DEM_E_CONTACT_OVERFLOW;
  return DEM_OK;
}

// With DEM_DEBUG set in the environment, a failed HIP call is named on
// stderr (the status code alone does not say which call failed).
void report_hip(hipError_t r, const char *expr, int line) {
  static const bool on = getenv("DEM_DEBUG") != nullptr;
  if (on) fprintf(stderr, "libdem: %s (line %d) failed: %s\n", expr, line, hipGetErrorString(r));
}

#define HIP_TRY(expr)                      \
  do {                                     \
    const hipError_t hip_r_ = (expr);      \
    if (hip_r_ != hipSuccess) {            \
      report_hip(hip_r_, #expr, __LINE__); \
      (void)hipGetLastError();             \
      return DEM_E_HIP;                    \
    }                                      \
  } while (0)

// Wait for the stream and fold the device error flags into the sticky status.
dem_status sync_and_check(Engine &e) {
  if (e.sticky != DEM_OK) {
    (void)hipStreamSynchronize(e.stream);
    return e.sticky;
  }
  int32_t bits = 0;
  if (hipMemcpyAsync(&bits, e.err, sizeof(int32_t), hipMemcpyDeviceToHost, e.stream) != hipSuccess ||
      hipStreamSynchronize(e.stream) != hipSuccess) {
    (void)hipGetLastError();
    e.sticky = DEM_E_HIP;
    return e.sticky;
  }
  e.sticky = map_err(bits);
  return e.sticky;
}

template <typename T>
dem_status d2h(Engine &e, const T *src, std::vector<T> &out, size_t count) {
  out.resize(count);
  if (count == 0) return DEM_OK;
  HIP_TRY(hipMemcpyAsync(out.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost, e.stream));
  HIP_TRY(hipStreamSynchronize(e.stream));
  return DEM_OK;
}

// `count` Reals from element `first` of a device array, as doubles
dem_status d2h_real(Engine &e, const void *src, size_t first, size_t count, std::vector<double> &out) {
  out.resize(count);
  if (count == 0) return DEM_OK;
  if (e.prec == DEM_PREC_FP64) {
    HIP_TRY(hipMemcpyAsync(out.data(), (const double *)src + first, sizeof(double) * count,
                           hipMemcpyDeviceToHost, e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
  } else {
    std::vector<float> tmp(count);
    HIP_TRY(hipMemcpyAsync(tmp.data(), (const float *)src + first, sizeof(float) * count, hipMemcpyDeviceToHost,
                           e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    for (size_t i = 0; i < count; i++) out[i] = (double)tmp[i];
  }
  return DEM_OK;
}

template <typename T>
dem_status h2d(Engine &e, T *dst, const std::vector<T> &src) {
  if (src.empty()) return DEM_OK;
  HIP_TRY(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, e.stream));
  HIP_TRY(hipStreamSynchronize(e.stream));
  return DEM_OK;
}

dem_status h2d_real(Engine &e, void *dst, const std::vector<double> &src) {
  if (src.empty()) return DEM_OK;
  if (e.prec == DEM_PREC_FP64) return h2d(e, (double *)dst, src);
  std::vector<float> tmp(src.size());
  for (size_t i = 0; i < src.size(); i++) tmp[i] = (float)src[i];
  return h2d(e, (float *)dst, tmp);
}

// component k of an n x 3 array in original order, arranged by slot
void gather3(const double *src, const std::vector<int32_t> &id_at_slot, int k, std::vector<double> &out) {
  out.resize(id_at_slot.size());
  for (size_t s = 0; s < id_at_slot.size(); s++) out[s] = src[3 * (size_t)id_at_slot[s] + k];
}

// Steps 5-8 detection on the current positions: the owned-contact lists
// (with ctl only the systems still stepping detect again; the others keep
// their lists)
hipError_t build_contacts(Engine &e, const StepCtl *ctl) {
  return launch_contacts(e.prec, e.layout(), ctl, e.nbr, e.scell, e.cell_start, nullptr, e.err, e.stream, nullptr);
}

// Steps 5-8 with the contact law (in the detection pass for the direct
// shape), then the per-particle sums (and, in a time step, the kicks)
hipError_t run_forces(Engine &e, const PairArgs &a, const StepCtl *ctl, hipEvent_t after_detect = nullptr,
                      hipEvent_t after_law = nullptr) {
  hipError_t r = launch_contacts(e.prec, a.L, ctl, e.nbr, e.scell, e.cell_start, &a, e.err, e.stream, after_detect);
  if (r != hipSuccess) return r;
  if (after_law) (void)hipEventRecord(after_law, e.stream);
  return launch_gather(e.prec, a, e.stream);
}

// Steps 7-8 on the current positions with the committed history of
// generation gc; a time step writes the new history into the other one
PairArgs pair_args(Engine &e, int mode, void *const F[3], void *const T[3]) {
  PairArgs a;
  memset(&a, 0, sizeof(a));
  a.L = e.layout();
  a.ctl = e.ctl;
  a.pos = e.pos[e.cp];
  a.pos_out = e.pos[e.cp ^ 1];
  a.vel_in = e.vel[e.cv];
  a.vel_out = e.vel[e.cv ^ 1];
  a.nb = e.nbr;
  a.cur = e.hist[e.gc ^ 1];
  a.old = e.hist[e.gc];
  a.w = e.work;
  for (int k = 0; k < 3; k++) {
    a.F[k] = F[k];
    a.T[k] = T[k];
  }
  a.diag = e.diag;
  a.cell = e.cell;
  a.scell = e.scell;
  a.cell_start = e.cell_start;
  a.mode = mode;
  a.law = e.law;
  a.terms = e.has_terms ? 1 : 0;
  a.mats = e.has_mt ? 1 : 0;
  a.err = e.err;
  return a;
}

struct Entry {
  int64_t a, b;
  double d[3];
};

// last slot + 1 of kernel block b
int32_t block_end(const Engine &e, size_t b) {
  const SysInfo &si = e.info[(size_t)e.bsys_h[b]];
  return std::min(e.bfirst_h[b] + kBlock, si.p0 + si.n);
}

// The history entries of generation g: counts and first entries per slot,
// and each block's entries (at most wmax of them, the most any block holds)
// as rows of wmax: delta_t (3 per entry, as doubles) and the keys (the bits
// of each entry's w).  Entry j of slot s of block b is at row b, column
// start[s] - cbase(b) + j.
dem_status read_hist_blocks(Engine &e, const HistGen &g, std::vector<int32_t> &cnt, std::vector<int32_t> &start,
                            size_t &wmax, std::vector<double> &d, std::vector<int32_t> &key) {
  const size_t N = (size_t)e.n, nb = e.bsys_h.size();
  dem_status st;
  if ((st = d2h(e, g.cnt, cnt, N)) != DEM_OK || (st = d2h(e, g.start, start, N)) != DEM_OK) return st;
  wmax = 0;
  for (size_t b = 0; b < nb; b++) {
    size_t tot = 0;
    for (int32_t sl = e.bfirst_h[b]; sl < block_end(e, b); sl++) tot += (size_t)std::min(std::max(cnt[sl], 0), e.K);
    wmax = std::max(wmax, tot);
  }
  const size_t m = wmax * nb;
  d.assign(3 * m, 0.0);
  key.assign(m, 0);
  if (m == 0) return DEM_OK;
  const size_t esz = 4 * e.rsz, spitch = (size_t)kBlock * e.K * esz;
  std::vector<char> raw(m * esz);
  HIP_TRY(hipMemcpy2DAsync(raw.data(), wmax * esz, g.ent, spitch, wmax * esz, nb, hipMemcpyDeviceToHost, e.stream));
  HIP_TRY(hipStreamSynchronize(e.stream));
  for (size_t q = 0; q < m; q++) {
    if (e.prec == DEM_PREC_FP64) {
      const double *r = (const double *)raw.data() + 4 * q;
      int64_t bits;
      memcpy(&bits, &r[3], 8);
      key[q] = (int32_t)bits;
      for (int c = 0; c < 3; c++) d[3 * q + c] = r[c];
    } else {
      const float *r = (const float *)raw.data() + 4 * q;
      memcpy(&key[q], &r[3], 4);
      for (int c = 0; c < 3; c++) d[3 * q + c] = (double)r[c];
    }
  }
  return DEM_OK;
}

// The contacts of system k as sorted (a, b) keys with ids local to the
// system: (lower id, higher id) for a pair, (id, -1 - w) for a wall.
// committed: the tangential history (with delta_t, turned to the view of the
// lower id); otherwise the owned-contact lists of the current positions.
dem_status read_gen(Engine &e, int32_t k, bool committed, std::vector<Entry> &out) {
  out.clear();
  const SysInfo &si = e.info[k];
  if (si.n == 0) return DEM_OK;
  const size_t N = (size_t)e.n;
  std::vector<int32_t> cnt, start, id, nb;
  std::vector<double> rows;
  std::vector<int32_t> keys;
  size_t wmax = 0;
  dem_status st;
  if (committed) {
    if ((st = read_hist_blocks(e, e.hist[e.gc], cnt, start, wmax, rows, keys)) != DEM_OK) return st;
  } else {
    if ((st = d2h(e, e.nbr.fcnt, cnt, N)) != DEM_OK) return st;
    int32_t kmax = 0;
    for (size_t slot = (size_t)si.p0; slot < (size_t)(si.p0 + si.n); slot++)
      kmax = std::max(kmax, std::min(std::max(cnt[slot], 0), e.K));
    if ((st = d2h(e, (const int32_t *)e.nbr.nb, nb, (size_t)kmax * N)) != DEM_OK) return st;
  }
  if ((st = d2h(e, (const int32_t *)e.pos[e.cp].id, id, N)) != DEM_OK) return st;
  for (size_t b = 0; b < e.bsys_h.size(); b++) {
    if (e.bsys_h[b] != k) continue;
    for (int32_t slot = e.bfirst_h[b]; slot < block_end(e, b); slot++) {
      const int32_t c = std::min(std::max(cnt[slot], 0), e.K);
      for (int32_t j = 0; j < c; j++) {
        const size_t q = committed ? b * wmax + (size_t)(start[slot] - cbase((int32_t)b, e.K)) + j
                                   : (size_t)j * N + (size_t)slot;
        Entry en;
        const int64_t me = id[slot] - si.p0;
        const int32_t other = committed ? keys[q] : nb[q];
        const bool pair = other >= 0;
        const int64_t them = pair ? id[other] - si.p0 : other;
        en.a = pair ? std::min(me, them) : me;
        en.b = pair ? std::max(me, them) : them;
        const double sg = (pair && me > them) ? -1.0 : 1.0;  // stored as seen from the owner slot
        for (int c3 = 0; c3 < 3; c3++) en.d[c3] = committed ? sg * rows[3 * q + c3] : 0.0;
        out.push_back(en);
      }
    }
  }
  std::sort(out.begin(), out.end(),
            [](const Entry &x, const Entry &y) { return x.a != y.a ? x.a < y.a : x.b < y.b; });
  return DEM_OK;
}

void free_graphs(Engine &e) {
  for (int p = 0; p < 2; p++) {
    if (e.gexec[p]) (void)hipGraphExecDestroy(e.gexec[p]);
    e.gexec[p] = nullptr;
    e.gexec_cp[p] = -1;
  }
}

void free_events(Engine &e) {
  for (hipEvent_t ev : e.events) (void)hipEventDestroy(ev);
  e.events.clear();
}

void release(Engine *e) {
  if (!e) return;
  (void)hipStreamSynchronize(e->stream);
  free_graphs(*e);
  free_events(*e);
  if (e->left_ev) (void)hipEventDestroy(e->left_ev);
  delete e;
}

// ----------------------------------------------------------------- create

struct HistIn {
  int64_t n = 0;
  const int64_t *pairs = nullptr;
  const double *dt = nullptr;
};

dem_status validate_inputs(Engine &e, const double *x, const double *v, const double *omega,
                           const double *r, const double *F0, const double *T0, const HistIn &hist,
                           std::vector<float> &rf) {
  const size_t N = (size_t)e.n;
  if (N > 0 && (!x || !v || !omega || !r)) return DEM_E_INVALID;
  // radii in FP32; the cell must hold the largest contact distance (27-cell search)
  rf.assign(N, 0.0f);
  for (int32_t k = 0; k < e.S; k++) {
    float rmax = 0.0f;
    SysInfo &si = e.info[k];
    for (int64_t i = si.p0; i < (int64_t)si.p0 + si.n; i++) {
      const float q = (float)r[i];
      if (!(q > 0.0f) || !isfinite(q)) return DEM_E_INVALID;
      rf[i] = q;
      rmax = std::max(rmax, q);
    }
    if (e.params[k].cell_size < 2.0 * (double)rmax) return DEM_E_INVALID;
    si.rmax = rmax;
  }
  for (size_t i = 0; i < 3 * N; i++)
    if (!isfinite(x[i]) || !isfinite(v[i]) || !isfinite(omega[i])) return DEM_E_NONFINITE;
  if (F0)
    for (size_t i = 0; i < 3 * N; i++)
      if (!isfinite(F0[i]) || !isfinite(T0[i])) return DEM_E_NONFINITE;
  if (e.law != DEM_LAW_SIMPLE) {
    // walls -1 .. -6 and plates -7 .. (a batch checked each system's own plates already)
    const int64_t wmin = -6 - (e.S == 1 ? e.params[0].nplates : kMaxPlates);
    for (int64_t k = 0; k < hist.n; k++) {
      const int64_t a = hist.pairs[2 * k], b = hist.pairs[2 * k + 1];
      const bool ok = a >= 0 && a < (int64_t)N && ((b > a && b < (int64_t)N) || (b < 0 && b >= wmin));
      if (!ok) return DEM_E_INVALID;
      for (int q = 0; q < 3; q++)
        if (!isfinite(hist.dt[3 * k + q])) return DEM_E_NONFINITE;
    }
  }
  return DEM_OK;
}

// The given history becomes generation 0: each contact filed under the lower
// slot of its pair (the particle for a wall) with delta_t seen from it, at
// [k * N + owner] for its k-th entry (keys ascending), with the owners'
// counts.  More entries for one particle than its capacity is an overflow.
dem_status upload_history(Engine &e, const HistIn &hist, const std::vector<int32_t> &id_at_slot) {
  const size_t N = (size_t)e.n;
  struct Rec {
    int32_t owner, key;
    double d[3];
  };
  std::vector<Rec> recs;
  if (e.law != DEM_LAW_SIMPLE && hist.n > 0) {
    std::vector<int32_t> slot_of(N);
    for (size_t sl = 0; sl < N; sl++) slot_of[id_at_slot[sl]] = (int32_t)sl;
    recs.reserve((size_t)hist.n);
    for (int64_t k = 0; k < hist.n; k++) {
      const int64_t a = hist.pairs[2 * k], b = hist.pairs[2 * k + 1];
      Rec rc;
      double sg = 1.0;
      if (b >= 0) {
        const int32_t sa = slot_of[a], sb = slot_of[b];
        rc.owner = std::min(sa, sb);
        rc.key = std::max(sa, sb);
        sg = sa < sb ? 1.0 : -1.0;  // given as seen from the lower id a
      } else {
        rc.owner = slot_of[a];
        rc.key = (int32_t)b;
      }
      for (int c = 0; c < 3; c++) rc.d[c] = sg * hist.dt[3 * k + c];
      recs.push_back(rc);
    }
    std::stable_sort(recs.begin(), recs.end(), [](const Rec &u, const Rec &w) {
      return u.owner != w.owner ? u.owner < w.owner : u.key < w.key;
    });
    for (size_t k = 1; k < recs.size(); k++)
      if (recs[k].owner == recs[k - 1].owner && recs[k].key == recs[k - 1].key) return DEM_E_INVALID;
  }
  std::vector<int32_t> cnt(N, 0);
  for (const Rec &rc : recs) cnt[rc.owner]++;
  for (size_t sl = 0; sl < N; sl++)
    if (cnt[sl] > e.info[e.psys_h[sl]].kcap) return DEM_E_CONTACT_OVERFLOW;
  // block layout: the entries of slot s of block b from cbase(b) + the
  // owned counts of the block's slots before s
  const size_t nb = e.bsys_h.size();
  std::vector<int32_t> start(N, 0);
  size_t wmax = 0;
  for (size_t b = 0; b < nb; b++) {
    int32_t run = 0;
    for (int32_t sl = e.bfirst_h[b]; sl < block_end(e, b); sl++) {
      start[sl] = (int32_t)cbase((int32_t)b, e.K) + run;
      run += cnt[sl];
    }
    wmax = std::max(wmax, (size_t)run);
  }
  const HistGen &g0 = e.hist[0];
  dem_status st;
  if ((st = h2d(e, g0.cnt, cnt)) != DEM_OK || (st = h2d(e, g0.start, start)) != DEM_OK) return st;
  if (recs.empty()) return DEM_OK;
  // entries: delta_t in x, y, z, the key's bits in w; one row of wmax per block
  std::vector<int32_t> blk(N, 0);
  for (size_t b = 0; b < nb; b++)
    for (int32_t sl = e.bfirst_h[b]; sl < block_end(e, b); sl++) blk[sl] = (int32_t)b;
  const size_t esz = 4 * e.rsz, m = wmax * nb;
  std::vector<char> raw(m * esz, 0);
  std::vector<int32_t> pos(N, 0);
  for (const Rec &rc : recs) {
    const int32_t b = blk[rc.owner];
    const size_t q = (size_t)b * wmax + (size_t)(start[rc.owner] - cbase(b, e.K)) + (size_t)pos[rc.owner]++;
    if (e.prec == DEM_PREC_FP64) {
      double *r = (double *)raw.data() + 4 * q;
      for (int c = 0; c < 3; c++) r[c] = rc.d[c];
      const int64_t bits = (int64_t)rc.key;
      memcpy(&r[3], &bits, 8);
    } else {
      float *r = (float *)raw.data() + 4 * q;
      for (int c = 0; c < 3; c++) r[c] = (float)rc.d[c];
      memcpy(&r[3], &rc.key, 4);
    }
  }
  HIP_TRY(hipMemcpy2DAsync(g0.ent, (size_t)kBlock * e.K * esz, raw.data(), wmax * esz, wmax * esz, nb,
                           hipMemcpyHostToDevice, e.stream));
  HIP_TRY(hipStreamSynchronize(e.stream));
  return DEM_OK;
}

dem_status engine_init(Engine &e, const double *x, const double *v, const double *omega,
                       const std::vector<float> &rf, const double *F0, const double *T0, const HistIn &hist) {
  const size_t N = (size_t)e.n;
  dem_status st;
  HIP_TRY(hipEventCreateWithFlags(&e.left_ev, hipEventDisableTiming));
  // tables
  std::vector<int32_t> zeros(64, 0);
  std::vector<int32_t> psys(N);
  for (int32_t k = 0; k < e.S; k++)
    for (int32_t i = 0; i < e.info[k].n; i++) psys[(size_t)e.info[k].p0 + i] = k;
  e.psys_h = psys;
  HIP_TRY(hipMemcpyAsync(e.tab, e.info.data(), sizeof(SysInfo) * e.info.size(), hipMemcpyHostToDevice, e.stream));
  HIP_TRY(hipStreamSynchronize(e.stream));
  if ((st = h2d(e, e.psys, psys)) != DEM_OK || (st = h2d(e, e.bsys, e.bsys_h)) != DEM_OK ||
      (st = h2d(e, e.tiles, e.tiles_h)) != DEM_OK || (st = h2d(e, e.runs, e.runs_h)) != DEM_OK ||
      (st = h2d(e, e.bfirst, e.bfirst_h)) != DEM_OK || (st = h2d(e, e.err, zeros)) != DEM_OK ||
      (st = h2d(e, e.ctl.step, zeros)) != DEM_OK)
    return st;
  // state in original order into buffer 0
  std::vector<int32_t> ids(N);
  std::iota(ids.begin(), ids.end(), 0);
  std::vector<double> tmp;
  double *dst[3] = {e.pos[0].x, e.pos[0].y, e.pos[0].z};
  for (int k = 0; k < 3; k++) {
    gather3(x, ids, k, tmp);
    if ((st = h2d(e, dst[k], tmp)) != DEM_OK) return st;
    gather3(v, ids, k, tmp);
    if ((st = h2d_real(e, e.vel[0].v[k], tmp)) != DEM_OK) return st;
    gather3(omega, ids, k, tmp);
    if ((st = h2d_real(e, e.vel[0].w[k], tmp)) != DEM_OK) return st;
  }
  if ((st = h2d(e, e.pos[0].r, rf)) != DEM_OK || (st = h2d(e, e.pos[0].id, ids)) != DEM_OK) return st;
  if (e.has_mt && (st = h2d(e, e.pos[0].mt, std::vector<int32_t>(N, 0))) != DEM_OK) return st;
  const Layout L = e.layout();
  // Steps 2-4 on the initial positions
  HIP_TRY(launch_hash(L, e.pos[0], e.cell, e.err, e.stream));
  HIP_TRY(launch_fill((int32_t *)e.reflag, (e.ncell + 3) / 4, 0, e.stream));
  HIP_TRY(launch_sort(e.cell, e.pos[0].id, nullptr, e.n, e.ncell, e.counts, e.rank, e.cell_start, e.perm,
                      e.reflag, e.scan, e.stream));
  HIP_TRY(launch_reorder(e.prec, L, e.pos[0], e.vel[0], e.pos[1], e.vel[1], true, e.perm, e.cell, e.scell, e.nbr,
                         nullptr, e.stream));
  e.cp = 1;
  e.cv = 1;
  e.gc = 0;
  // no backward contact is filed yet (each gather clears its count)
  HIP_TRY(launch_fill(e.work.nback, (int64_t)e.bfirst_h.size(), 0, e.stream));
  // Steps 5-6: the contacts of the initial positions
  HIP_TRY(build_contacts(e, nullptr));
  if ((st = sync_and_check(e)) != DEM_OK) return st;
  std::vector<int32_t> id_at_slot;
  if ((st = d2h(e, e.pos[1].id, id_at_slot, N)) != DEM_OK) return st;
  if ((st = upload_history(e, hist, id_at_slot)) != DEM_OK) return st;
  // forces of the initial state: given, or evaluated with the given history
  if (F0) {
    for (int k = 0; k < 3; k++) {
      gather3(F0, id_at_slot, k, tmp);
      if ((st = h2d_real(e, e.F[k], tmp)) != DEM_OK) return st;
      gather3(T0, id_at_slot, k, tmp);
      if ((st = h2d_real(e, e.T[k], tmp)) != DEM_OK) return st;
    }
  } else {
    PairArgs a = pair_args(e, 0, e.F, e.T);
    HIP_TRY(run_forces(e, a, nullptr));
  }
  return sync_and_check(e);
}

dem_status engine_create(int32_t S, const dem_params *p, const int64_t *n, const double *x, const double *v,
                         const double *omega, const double *r, const double *F0, const double *T0,
                         const HistIn &hist, void *workspace, size_t ws_bytes, void *hip_stream, Engine **out) {
  *out = nullptr;
  Engine *e = new (std::nothrow) Engine;
  if (!e) return DEM_E_INVALID;
  dem_status st = plan(*e, S, p, n);
  std::vector<float> rf;
  if (st == DEM_OK) st = validate_inputs(*e, x, v, omega, r, F0, T0, hist, rf);
  if (st == DEM_OK) {
    const size_t need = carve(*e, nullptr);
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255)) st = DEM_E_WORKSPACE;
  }
  if (st != DEM_OK) {
    delete e;
    return st;
  }
  e->stream = (hipStream_t)hip_stream;
  // an error another library left on this thread is not ours: the launches
  // below check hipGetLastError after each kernel
  (void)hipGetLastError();
  carve(*e, (char *)workspace);
  st = engine_init(*e, x, v, omega, rf, F0, T0, hist);
  if (st != DEM_OK) {
    release(e);
    return st;
  }
  *out = e;
  return DEM_OK;
}

// ----------------------------------------------------------------- step

// Steps 3-8 of one time step.  Steps 1-2 (opening kick, drift, hash) run
// before the first step of a call and, after that, inside the previous
// step's gather for every system that steps again.  The reorder moves the
// state to the other buffers and the gather moves it back, so a step starts
// from the same buffers every time.
hipError_t step_body(Engine &e, hipEvent_t *ev) {
  auto mark = [&](int phase) {
    if (ev) (void)hipEventRecord(ev[phase], e.stream);
  };
  const Layout L = e.layout();
  hipError_t r;
  // Step 3
  if ((r = launch_sort(e.cell, e.pos[e.cp].id, e.scell, e.n, e.ncell, e.counts, e.rank, e.cell_start, e.perm,
                       e.reflag, e.scan, e.stream)) != hipSuccess)
    return r;
  mark(2);
  // Step 4
  // (the state goes into the packed records only; the gather writes it back)
  if ((r = launch_reorder(e.prec, L, e.pos[e.cp], e.vel[e.cv], e.pos[e.cp ^ 1], e.vel[e.cv ^ 1], false, e.perm,
                          e.cell, e.scell, e.nbr, &e.hist[e.gc], e.stream)) != hipSuccess)
    return r;
  e.cp ^= 1;
  e.cv ^= 1;
  mark(3);
  // Steps 5-8 and the closing half kick; the new history goes into the
  // generation that does not hold the committed one, and is committed
  PairArgs a = pair_args(e, MODE_WRITE_HIST | MODE_KICK | MODE_OLD_PERM, e.F, e.T);
  if ((r = run_forces(e, a, &e.ctl, ev ? ev[4] : nullptr, ev ? ev[5] : nullptr)) != hipSuccess) return r;
  if ((r = launch_step_end(e.ctl, e.stream)) != hipSuccess) return r;
  mark(6);
  e.cp ^= 1;
  e.cv ^= 1;
  e.gc ^= 1;
  return hipSuccess;
}

// Capture the step body for the current history generation.  Every argument
// of every launch is fixed by (cp, cv, gc); cp and cv are the same at the
// start of every step, so one graph per gc replays every later step.
dem_status capture(Engine &e) {
  const int cp = e.cp, cv = e.cv, gc = e.gc;
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(e.stream, hipStreamCaptureModeThreadLocal));
  const hipError_t r = step_body(e, nullptr);
  const hipError_t r2 = hipStreamEndCapture(e.stream, &graph);
  e.cp = cp;
  e.cv = cv;
  e.gc = gc;
  if (r != hipSuccess || r2 != hipSuccess || !graph) {
    (void)hipGetLastError();
    if (graph) (void)hipGraphDestroy(graph);
    return DEM_E_HIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t r3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (r3 != hipSuccess) {
    (void)hipGetLastError();
    return DEM_E_HIP;
  }
  if (e.gexec[gc]) (void)hipGraphExecDestroy(e.gexec[gc]);
  e.gexec[gc] = exec;
  e.gexec_cp[gc] = cp | (cv << 1);
  return DEM_OK;
}

dem_status engine_step(Engine &e, const int64_t *steps) {
  if (e.sticky != DEM_OK) return e.sticky;
  int64_t maxs = 0;
  for (int32_t k = 0; k < e.S; k++) {
    if (steps[k] < 0 || steps[k] > (int64_t)INT32_MAX / 2) return DEM_E_INVALID;
    maxs = std::max(maxs, steps[k]);
  }
  if (maxs == 0) return DEM_OK;
  (void)hipGetLastError();  // not ours (see engine_create)
  // the previous call's upload of left[] must have been read before the
  // host array is overwritten
  if (e.left_pending && hipEventSynchronize(e.left_ev) != hipSuccess) return e.sticky = DEM_E_HIP;
  for (int32_t k = 0; k < e.S; k++) e.left_h[k] = (int32_t)steps[k];
  if (hipMemcpyAsync(e.ctl.left, e.left_h.data(), sizeof(int32_t) * e.S, hipMemcpyHostToDevice, e.stream) !=
          hipSuccess ||
      hipEventRecord(e.left_ev, e.stream) != hipSuccess || launch_fill(e.ctl.step, 1, 0, e.stream) != hipSuccess) {
    (void)hipGetLastError();
    return e.sticky = DEM_E_HIP;
  }
  e.left_pending = true;
  const Layout L = e.layout();
  for (int64_t k = 0; k < maxs; k++) {
    hipEvent_t *ev = nullptr;
    if (e.profiling && e.timed < DEM_PROFILE_CAPACITY) {
      ev = e.events.data() + (size_t)e.timed * (DEM_NUM_PHASES + 1);
      e.timed++;
    }
    if (ev) (void)hipEventRecord(ev[0], e.stream);
    // Steps 1-2 for the first step of the call
    if (k == 0 && launch_kick_drift_hash(e.prec, L, e.ctl, e.pos[e.cp], e.vel[e.cv], e.F, e.T, e.scell, e.cell,
                                         e.err, e.stream) != hipSuccess) {
      (void)hipGetLastError();
      return e.sticky = DEM_E_HIP;
    }
    if (ev) (void)hipEventRecord(ev[1], e.stream);
    if (e.use_graph) {
      const int par = e.gc;
      if (!e.gexec[par] || e.gexec_cp[par] != (e.cp | (e.cv << 1))) {
        const dem_status st = capture(e);
        if (st != DEM_OK) return e.sticky = st;
      }
      if (ev)
        for (int p = 2; p < DEM_NUM_PHASES; p++) (void)hipEventRecord(ev[p], e.stream);
      if (hipGraphLaunch(e.gexec[par], e.stream) != hipSuccess) {
        (void)hipGetLastError();
        return e.sticky = DEM_E_HIP;
      }
      if (ev) (void)hipEventRecord(ev[DEM_NUM_PHASES], e.stream);
      // what the replayed body does to the indices (cp and cv come back)
      e.gc ^= 1;
    } else if (step_body(e, ev) != hipSuccess) {
      (void)hipGetLastError();
      return e.sticky = DEM_E_HIP;
    }
  }
  return DEM_OK;
}

dem_status engine_use_graph(Engine &e, int enable) {
  if (enable && e.stream == nullptr) return DEM_E_INVALID;  // no capture on the null stream
  HIP_TRY(hipStreamSynchronize(e.stream));
  e.use_graph = enable != 0;
  if (!e.use_graph) free_graphs(e);
  return DEM_OK;
}

dem_status engine_forces(Engine &e, double *F, double *T) {
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  PairArgs a = pair_args(e, 0, e.Fe, e.Te);
  if (launch_pack(e.prec, e.layout(), e.pos[e.cp], e.vel[e.cv], e.nbr, e.stream) != hipSuccess ||
      run_forces(e, a, nullptr) != hipSuccess) {
    (void)hipGetLastError();
    return e.sticky = DEM_E_HIP;
  }
  if ((st = sync_and_check(e)) != DEM_OK) return st;
  const size_t N = (size_t)e.n;
  std::vector<int32_t> id;
  if ((st = d2h(e, e.pos[e.cp].id, id, N)) != DEM_OK) return st;
  std::vector<double> tmp;
  for (int k = 0; k < 3; k++) {
    if ((st = d2h_real(e, e.Fe[k], 0, N, tmp)) != DEM_OK) return st;
    for (size_t i = 0; i < N; i++) F[3 * (size_t)id[i] + k] = tmp[i];
    if ((st = d2h_real(e, e.Te[k], 0, N, tmp)) != DEM_OK) return st;
    for (size_t i = 0; i < N; i++) T[3 * (size_t)id[i] + k] = tmp[i];
  }
  return DEM_OK;
}

// state of system k, in the system's own original order
dem_status engine_read_state(Engine &e, int32_t k, double *x, double *v, double *omega, double *F, double *T) {
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  const SysInfo &si = e.info[k];
  const size_t p0 = (size_t)si.p0, n = (size_t)si.n;
  std::vector<int32_t> id;
  if ((st = d2h(e, e.pos[e.cp].id + p0, id, n)) != DEM_OK) return st;
  for (size_t i = 0; i < n; i++) id[i] -= (int32_t)p0;
  std::vector<double> tmp;
  if (x) {
    const double *src[3] = {e.pos[e.cp].x, e.pos[e.cp].y, e.pos[e.cp].z};
    for (int c = 0; c < 3; c++) {
      if ((st = d2h(e, src[c] + p0, tmp, n)) != DEM_OK) return st;
      for (size_t i = 0; i < n; i++) x[3 * (size_t)id[i] + c] = tmp[i];
    }
  }
  void *const *arrs[4] = {e.vel[e.cv].v, e.vel[e.cv].w, e.F, e.T};
  double *outs[4] = {v, omega, F, T};
  for (int q = 0; q < 4; q++) {
    if (!outs[q]) continue;
    for (int c = 0; c < 3; c++) {
      if ((st = d2h_real(e, arrs[q][c], p0, n, tmp)) != DEM_OK) return st;
      for (size_t i = 0; i < n; i++) outs[q][3 * (size_t)id[i] + c] = tmp[i];
    }
  }
  return DEM_OK;
}

// committed: the tangential history; otherwise the contacts of the current
// positions (keys only)
dem_status engine_read_contacts(Engine &e, int32_t k, bool committed, int64_t cap, int64_t *n_out,
                                int64_t *pairs, double *delta_t) {
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  std::vector<Entry> ent;
  if (!(committed && e.law == DEM_LAW_SIMPLE) && (st = read_gen(e, k, committed, ent)) != DEM_OK) return st;
  *n_out = (int64_t)ent.size();
  if ((int64_t)ent.size() > cap) return DEM_E_CAPACITY;
  for (size_t q = 0; q < ent.size(); q++) {
    if (pairs) {
      pairs[2 * q] = ent[q].a;
      pairs[2 * q + 1] = ent[q].b;
    }
    if (delta_t)
      for (int c = 0; c < 3; c++) delta_t[3 * q + c] = ent[q].d[c];
  }
  return DEM_OK;
}

dem_status engine_diagnostics(Engine &e, double *out) {
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  PairArgs a = pair_args(e, MODE_DIAG, e.Fe, e.Te);
  if (launch_pack(e.prec, e.layout(), e.pos[e.cp], e.vel[e.cv], e.nbr, e.stream) != hipSuccess ||
      run_forces(e, a, nullptr) != hipSuccess ||
      launch_diag_reduce(e.prec, e.layout(), e.pos[e.cp], e.vel[e.cv], e.diag, e.stream) != hipSuccess) {
    (void)hipGetLastError();
    return e.sticky = DEM_E_HIP;
  }
  if ((st = sync_and_check(e)) != DEM_OK) return st;
  std::vector<double> o;
  if ((st = d2h(e, (const double *)e.diag.out, o, 10 * (size_t)e.S)) != DEM_OK) return st;
  memcpy(out, o.data(), o.size() * sizeof(double));
  return DEM_OK;
}

// Replace the radii of every system (the engine's original order: systems
// concatenated), then rebuild the contact list beside the committed history.
dem_status engine_set_radii(Engine &e, const double *r) {
  if (e.n > 0 && !r) return DEM_E_INVALID;
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  const size_t N = (size_t)e.n;
  std::vector<float> rf(N);
  std::vector<SysInfo> info = e.info;
  for (int32_t k = 0; k < e.S; k++) {
    double rmax = 0.0;
    for (int64_t i = info[k].p0; i < (int64_t)info[k].p0 + info[k].n; i++) {
      const float q = (float)r[i];
      if (!(q > 0.0f) || !isfinite(q)) return DEM_E_INVALID;
      rf[i] = q;
      rmax = std::max(rmax, (double)q);
    }
    if (e.params[k].cell_size < 2.0 * rmax) return DEM_E_INVALID;
    info[k].rmax = (float)rmax;
  }
  if (N == 0) return DEM_OK;
  e.info = info;
  HIP_TRY(hipMemcpyAsync(e.tab, e.info.data(), sizeof(SysInfo) * e.info.size(), hipMemcpyHostToDevice, e.stream));
  HIP_TRY(hipStreamSynchronize(e.stream));
  std::vector<int32_t> id;
  if ((st = d2h(e, e.pos[e.cp].id, id, N)) != DEM_OK) return st;
  std::vector<float> slot_r(N);
  for (size_t k = 0; k < N; k++) slot_r[k] = rf[id[k]];
  if ((st = h2d(e, e.pos[e.cp].r, slot_r)) != DEM_OK) return st;
  HIP_TRY(launch_xyzr(e.layout(), e.pos[e.cp], e.nbr, e.stream));
  HIP_TRY(launch_pack(e.prec, e.layout(), e.pos[e.cp], e.vel[e.cv], e.nbr, e.stream));
  // the contact list of the new radii, beside the committed history
  HIP_TRY(build_contacts(e, nullptr));
  return sync_and_check(e);
}

// Material-pair table of system k (Sec. 3, the (i, j) constants of Eqs. 8-10;
// ntypes = 0: back to the system's one material), then the stored forces of
// system k evaluated again on its current state with the committed history.
dem_status engine_set_materials(Engine &e, int32_t k, int32_t ntypes, const double *table, const int32_t *type,
                                int32_t wall_type) {
  if (k < 0 || k >= e.S) return DEM_E_INVALID;
  const dem_params &p = e.params[k];
  SysInfo si = e.info[k];
  const size_t n = (size_t)si.n, p0 = (size_t)si.p0;
  if (ntypes < 0 || ntypes > p.max_materials) return DEM_E_INVALID;
  std::vector<PairK> tab((size_t)ntypes * ntypes);
  if (ntypes > 0) {
    if (!table || (n > 0 && !type) || wall_type < 0 || wall_type >= ntypes) return DEM_E_INVALID;
    for (int32_t t = 0; t < ntypes; t++)
      for (int32_t u = 0; u < ntypes; u++) {
        const double *q = table + 4 * ((size_t)t * ntypes + u), *qt = table + 4 * ((size_t)u * ntypes + t);
        if (!(q[0] > 0.0) || !(q[1] >= 0.0) || !(q[2] > 0.0 && q[2] <= 1.0) || !(q[3] >= 0.0) ||
            !isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[3]))
          return DEM_E_INVALID;
        for (int c = 0; c < 4; c++)
          if (q[c] != qt[c]) return DEM_E_INVALID;
        tab[(size_t)t * ntypes + u] = PairK{q[0], q[1], alpha_of(q[2]), q[3]};
      }
    for (size_t i = 0; i < n; i++)
      if (type[i] < 0 || type[i] >= ntypes) return DEM_E_INVALID;
  }
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  if (n == 0 || !e.has_mt) {
    e.info[k].ntypes = ntypes;
    e.info[k].wall_type = ntypes > 0 ? wall_type : 0;
    return DEM_OK;
  }
  // materials of the system's slots
  std::vector<int32_t> id;
  if ((st = d2h(e, e.pos[e.cp].id + p0, id, n)) != DEM_OK) return st;
  std::vector<int32_t> slot_t(n, 0);
  if (ntypes > 0)
    for (size_t j = 0; j < n; j++) slot_t[j] = type[(size_t)id[j] - p0];
  if ((st = h2d(e, e.pos[e.cp].mt + p0, slot_t)) != DEM_OK) return st;
  if (ntypes > 0) HIP_TRY(hipMemcpyAsync(e.mat + si.mat0, tab.data(), sizeof(PairK) * tab.size(),
                                         hipMemcpyHostToDevice, e.stream));
  si.ntypes = ntypes;
  si.wall_type = ntypes > 0 ? wall_type : 0;
  e.info[k] = si;
  HIP_TRY(hipMemcpyAsync(e.tab + k, &e.info[k], sizeof(SysInfo), hipMemcpyHostToDevice, e.stream));
  // forces of every system into the scratch force arrays; system k's become
  // its stored forces (the others keep theirs)
  PairArgs a = pair_args(e, 0, e.Fe, e.Te);
  HIP_TRY(launch_pack(e.prec, e.layout(), e.pos[e.cp], e.vel[e.cv], e.nbr, e.stream));
  HIP_TRY(run_forces(e, a, nullptr));
  for (int c = 0; c < 3; c++) {
    HIP_TRY(hipMemcpyAsync((char *)e.F[c] + e.rsz * p0, (const char *)e.Fe[c] + e.rsz * p0, e.rsz * n,
                           hipMemcpyDeviceToDevice, e.stream));
    HIP_TRY(hipMemcpyAsync((char *)e.T[c] + e.rsz * p0, (const char *)e.Te[c] + e.rsz * p0, e.rsz * n,
                           hipMemcpyDeviceToDevice, e.stream));
  }
  return sync_and_check(e);
}

// largest |v| of every system's current state
dem_status engine_max_speed(Engine &e, std::vector<double> &out) {
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  HIP_TRY(launch_fill((int32_t *)e.vmax, 2 * (int64_t)e.S, 0, e.stream));
  HIP_TRY(launch_max_speed(e.prec, e.layout(), e.vel[e.cv], e.vmax, e.stream));
  std::vector<unsigned long long> bits;
  if ((st = d2h(e, e.vmax, bits, (size_t)e.S)) != DEM_OK) return st;
  out.resize((size_t)e.S);
  for (int32_t k = 0; k < e.S; k++) memcpy(&out[k], &bits[k], sizeof(double));
  return DEM_OK;
}

dem_status engine_profile(Engine &e, int enable) {
  if (enable && e.events.empty()) {
    const size_t cnt = (size_t)DEM_PROFILE_CAPACITY * (DEM_NUM_PHASES + 1);
    e.events.assign(cnt, nullptr);
    for (size_t k = 0; k < cnt; k++)
      if (hipEventCreate(&e.events[k]) != hipSuccess) {
        (void)hipGetLastError();
        e.events.resize(k);
        free_events(e);
        return DEM_E_HIP;
      }
  }
  e.profiling = enable != 0;
  e.timed = 0;
  return DEM_OK;
}

dem_status engine_profile_read(Engine &e, double ms[DEM_NUM_PHASES], int64_t *steps) {
  HIP_TRY(hipStreamSynchronize(e.stream));
  for (int p = 0; p < DEM_NUM_PHASES; p++) ms[p] = 0.0;
  for (int64_t k = 0; k < e.timed; k++) {
    hipEvent_t *ev = e.events.data() + (size_t)k * (DEM_NUM_PHASES + 1);
    for (int p = 0; p < DEM_NUM_PHASES; p++) {
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, ev[p], ev[p + 1]));
      ms[p] += (double)t;
    }
  }
  *steps = e.timed;
  e.timed = 0;
  return DEM_OK;
}

}  // namespace

struct dem_system {
  Engine *e;
  int static_dev = -1;  // device whose static workspace it uses (dem_create_static), else -1
};

// The workspace of systems made by dem_create_static, for callers that
// cannot allocate device memory: one array per device, loaded with the code
// object and held until the process ends.  On the host the array's name is
// only a stand-in for the device symbol, never an address: the device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current and kept per device, and only that address is handed to
// the kernels (through the same carving as a caller's workspace).
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {
constexpr int kMaxDevices = 64;
struct StaticSlot {
  void *ptr = nullptr;                // device address of the array on this device
  const dem_system *owner = nullptr;  // the live system that uses it
};
std::mutex g_static_mu;
StaticSlot g_static[kMaxDevices];
}  // namespace
struct dem_batch {
  Engine *e;
};

extern "C" {

const char *dem_status_string(dem_status st) {
  switch (st) {
    case DEM_OK: return "ok";
    case DEM_E_INVALID: return "invalid argument";
    case DEM_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case DEM_E_CONTACT_OVERFLOW: return "contact list overflow";
    case DEM_E_OUT_OF_DOMAIN: return "particle out of domain";
    case DEM_E_NONFINITE: return "non-finite state or force";
    case DEM_E_HIP: return "HIP runtime error";
    case DEM_E_STATE: return "handle unusable";
    case DEM_E_CAPACITY: return "output capacity too small";
  }
  return "unknown status";
}

// ----------------------------------------------------------------- one system

dem_status dem_workspace_bytes(const dem_params *p, int64_t n, size_t *bytes) {
  return dem_batch_workspace_bytes(1, p, &n, bytes);
}

dem_status dem_create(const dem_params *p, int64_t n, const double *x, const double *v, const double *omega,
                      const double *r, const double *F0, const double *T0, int64_t n_hist,
                      const int64_t *hist_pairs, const double *hist_dt, void *workspace, size_t ws_bytes,
                      void *hip_stream, dem_system **out) {
  if (!out) return DEM_E_INVALID;
  *out = nullptr;
  if ((F0 == nullptr) != (T0 == nullptr)) return DEM_E_INVALID;
  if (n_hist < 0 || (n_hist > 0 && (!hist_pairs || !hist_dt))) return DEM_E_INVALID;
  HistIn h;
  h.n = n_hist;
  h.pairs = hist_pairs;
  h.dt = hist_dt;
  Engine *e = nullptr;
  const dem_status st = engine_create(1, p, &n, x, v, omega, r, F0, T0, h, workspace, ws_bytes, hip_stream, &e);
  if (st != DEM_OK) return st;
  dem_system *s = new (std::nothrow) dem_system;
  if (!s) {
    release(e);
    return DEM_E_INVALID;
  }
  s->e = e;
  *out = s;
  return DEM_OK;
}

size_t dem_static_workspace_capacity(void) { return kStaticWorkspaceBytes; }

dem_status dem_create_static(const dem_params *p, int64_t n, const double *x, const double *v,
                             const double *omega, const double *r, const double *F0, const double *T0,
                             int64_t n_hist, const int64_t *hist_pairs, const double *hist_dt, void *hip_stream,
                             dem_system **out) {
  if (!out) return DEM_E_INVALID;
  *out = nullptr;
  size_t need = 0;
  dem_status st = dem_workspace_bytes(p, n, &need);
  if (st != DEM_OK) return st;
  if (need > kStaticWorkspaceBytes) return DEM_E_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return DEM_E_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return DEM_E_INVALID;
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot &slot = g_static[dev];
  if (slot.owner) return DEM_E_STATE;  // the device's array is in use
  if (!slot.ptr) {
    void *ptr = nullptr;
    const hipError_t r = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (r != hipSuccess || !ptr) {
      report_hip(r, "hipGetSymbolAddress(scratch)", __LINE__);
      (void)hipGetLastError();
      return DEM_E_HIP;
    }
    slot.ptr = ptr;
  }
  st = dem_create(p, n, x, v, omega, r, F0, T0, n_hist, hist_pairs, hist_dt, slot.ptr, kStaticWorkspaceBytes,
                  hip_stream, out);
  if (st != DEM_OK) return st;
  (*out)->static_dev = dev;
  slot.owner = *out;
  return DEM_OK;
}

dem_status dem_step(dem_system *s, int64_t nsteps) {
  if (!s) return DEM_E_STATE;
  return engine_step(*s->e, &nsteps);
}

dem_status dem_sync(dem_system *s) {
  if (!s) return DEM_E_STATE;
  return sync_and_check(*s->e);
}

dem_status dem_use_graph(dem_system *s, int enable) {
  if (!s) return DEM_E_STATE;
  return engine_use_graph(*s->e, enable);
}

dem_status dem_forces(dem_system *s, double *F, double *T) {
  if (!s) return DEM_E_STATE;
  if (s->e->n > 0 && (!F || !T)) return DEM_E_INVALID;
  return engine_forces(*s->e, F, T);
}

dem_status dem_read_state(dem_system *s, double *x, double *v, double *omega, double *F, double *T) {
  if (!s) return DEM_E_STATE;
  return engine_read_state(*s->e, 0, x, v, omega, F, T);
}

dem_status dem_read_contacts(dem_system *s, int64_t cap, int64_t *n_out, int64_t *pairs, double *delta_t) {
  if (!s) return DEM_E_STATE;
  if (!n_out) return DEM_E_INVALID;
  return engine_read_contacts(*s->e, 0, true, cap, n_out, pairs, delta_t);
}

dem_status dem_contacts(dem_system *s, int64_t cap, int64_t *n_out, int64_t *pairs) {
  if (!s) return DEM_E_STATE;
  if (!n_out) return DEM_E_INVALID;
  return engine_read_contacts(*s->e, 0, false, cap, n_out, pairs, nullptr);
}

dem_status dem_read_grid(dem_system *s, int32_t *cell_of_id, int32_t *id_at_slot, int32_t *cell_start) {
  if (!s) return DEM_E_STATE;
  Engine &e = *s->e;
  dem_status st = sync_and_check(e);
  if (st != DEM_OK) return st;
  const size_t N = (size_t)e.n;
  std::vector<int32_t> id, sc;
  if ((st = d2h(e, e.pos[e.cp].id, id, N)) != DEM_OK) return st;
  if (cell_of_id) {
    if ((st = d2h(e, (const int32_t *)e.scell, sc, N)) != DEM_OK) return st;
    for (size_t i = 0; i < N; i++) cell_of_id[id[i]] = sc[i];
  }
  if (id_at_slot && N) memcpy(id_at_slot, id.data(), 4 * N);
  if (cell_start) {
    std::vector<int32_t> cs;
    if ((st = d2h(e, (const int32_t *)e.cell_start, cs, (size_t)e.ncell + 1)) != DEM_OK) return st;
    memcpy(cell_start, cs.data(), 4 * cs.size());
  }
  return DEM_OK;
}

dem_status dem_grid_dims(dem_system *s, int32_t dims[3]) {
  if (!s) return DEM_E_STATE;
  if (!dims) return DEM_E_INVALID;
  for (int a = 0; a < 3; a++) dims[a] = s->e->info[0].g.nc[a];
  return DEM_OK;
}

dem_status dem_diagnostics(dem_system *s, double out[10]) {
  if (!s) return DEM_E_STATE;
  if (!out) return DEM_E_INVALID;
  return engine_diagnostics(*s->e, out);
}

dem_status dem_set_radii(dem_system *s, const double *r) {
  if (!s) return DEM_E_STATE;
  return engine_set_radii(*s->e, r);
}

dem_status dem_set_materials(dem_system *s, int32_t ntypes, const double *table, const int32_t *type,
                             int32_t wall_type) {
  if (!s) return DEM_E_STATE;
  return engine_set_materials(*s->e, 0, ntypes, table, type, wall_type);
}

dem_status dem_max_speed(dem_system *s, double *vmax) {
  if (!s) return DEM_E_STATE;
  if (!vmax) return DEM_E_INVALID;
  std::vector<double> out;
  const dem_status st = engine_max_speed(*s->e, out);
  if (st == DEM_OK) *vmax = out[0];
  return st;
}

dem_status dem_run_to_rest(dem_system *s, double threshold, int64_t check_every, int64_t max_steps,
                           int64_t *steps_done) {
  if (!s) return DEM_E_STATE;
  if (!steps_done || !(threshold >= 0.0) || check_every < 1 || max_steps < 0) return DEM_E_INVALID;
  *steps_done = 0;
  const double dt = s->e->params[0].dt;
  while (*steps_done < max_steps) {
    const int64_t k = std::min(check_every, max_steps - *steps_done);
    dem_status st = engine_step(*s->e, &k);
    if (st != DEM_OK) return st;
    *steps_done += k;
    double vmax = 0.0;
    if ((st = dem_max_speed(s, &vmax)) != DEM_OK) return st;
    if (dt * vmax < threshold) break;
  }
  return DEM_OK;
}

dem_status dem_profile(dem_system *s, int enable) {
  if (!s) return DEM_E_STATE;
  return engine_profile(*s->e, enable);
}

dem_status dem_profile_read(dem_system *s, double ms[DEM_NUM_PHASES], int64_t *steps) {
  if (!s) return DEM_E_STATE;
  if (!ms || !steps) return DEM_E_INVALID;
  return engine_profile_read(*s->e, ms, steps);
}

dem_status dem_destroy(dem_system *s) {
  if (!s) return DEM_E_STATE;
  release(s->e);  // waits for the stream: nothing of the system runs after this
  if (s->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static[s->static_dev].owner == s) g_static[s->static_dev].owner = nullptr;
  }
  delete s;
  return DEM_OK;
}

// ----------------------------------------------------------------- batches

dem_status dem_batch_workspace_bytes(int32_t n_sys, const dem_params *p, const int64_t *n, size_t *bytes) {
  if (!bytes) return DEM_E_INVALID;
  Engine e;
  const dem_status st = plan(e, n_sys, p, n);
  if (st != DEM_OK) return st;
  *bytes = carve(e, nullptr);
  return DEM_OK;
}

dem_status dem_batch_create(int32_t n_sys, const dem_params *p, const int64_t *n, const double *x,
                            const double *v, const double *omega, const double *r, const double *F0,
                            const double *T0, const int64_t *n_hist, const int64_t *hist_pairs,
                            const double *hist_dt, void *workspace, size_t ws_bytes, void *hip_stream,
                            dem_batch **out) {
  if (!out) return DEM_E_INVALID;
  *out = nullptr;
  if ((F0 == nullptr) != (T0 == nullptr) || n_sys < 1 || !n) return DEM_E_INVALID;
  // the systems' history keys (local ids) become keys over the whole batch
  std::vector<int64_t> gpairs;
  HistIn h;
  if (n_hist) {
    int64_t tot = 0, base = 0;
    for (int32_t k = 0; k < n_sys; k++) {
      if (n_hist[k] < 0 || n[k] < 0) return DEM_E_INVALID;
      tot += n_hist[k];
    }
    if (tot > 0 && (!hist_pairs || !hist_dt)) return DEM_E_INVALID;
    gpairs.resize((size_t)(2 * tot));
    int64_t q = 0;
    for (int32_t k = 0; k < n_sys; k++) {
      for (int64_t j = 0; j < n_hist[k]; j++, q++) {
        const int64_t a = hist_pairs[2 * q], b = hist_pairs[2 * q + 1];
        const bool ok = a >= 0 && a < n[k] && ((b > a && b < n[k]) || (b < 0 && b >= -6 - p[k].nplates));
        if (!ok) return DEM_E_INVALID;
        gpairs[2 * q] = a + base;
        gpairs[2 * q + 1] = b >= 0 ? b + base : b;
      }
      base += n[k];
    }
    h.n = tot;
    h.pairs = gpairs.data();
    h.dt = hist_dt;
  }
  Engine *e = nullptr;
  const dem_status st = engine_create(n_sys, p, n, x, v, omega, r, F0, T0, h, workspace, ws_bytes, hip_stream, &e);
  if (st != DEM_OK) return st;
  dem_batch *b = new (std::nothrow) dem_batch;
  if (!b) {
    release(e);
    return DEM_E_INVALID;
  }
  b->e = e;
  *out = b;
  return DEM_OK;
}

dem_status dem_batch_set_materials(dem_batch *b, int32_t k, int32_t ntypes, const double *table,
                                   const int32_t *type, int32_t wall_type) {
  if (!b) return DEM_E_STATE;
  return engine_set_materials(*b->e, k, ntypes, table, type, wall_type);
}

dem_status dem_batch_max_speed(dem_batch *b, double *vmax) {
  if (!b) return DEM_E_STATE;
  if (!vmax) return DEM_E_INVALID;
  std::vector<double> out;
  const dem_status st = engine_max_speed(*b->e, out);
  if (st == DEM_OK) memcpy(vmax, out.data(), sizeof(double) * out.size());
  return st;
}

dem_status dem_batch_step(dem_batch *b, const int64_t *steps) {
  if (!b) return DEM_E_STATE;
  if (!steps) return DEM_E_INVALID;
  return engine_step(*b->e, steps);
}

dem_status dem_batch_set_radii(dem_batch *b, const double *r) {
  if (!b) return DEM_E_STATE;
  return engine_set_radii(*b->e, r);
}

dem_status dem_batch_read_state(dem_batch *b, int32_t k, double *x, double *v, double *omega, double *F,
                                double *T) {
  if (!b) return DEM_E_STATE;
  if (k < 0 || k >= b->e->S) return DEM_E_INVALID;
  return engine_read_state(*b->e, k, x, v, omega, F, T);
}

dem_status dem_batch_read_contacts(dem_batch *b, int32_t k, int64_t cap, int64_t *n_out, int64_t *pairs,
                                   double *delta_t) {
  if (!b) return DEM_E_STATE;
  if (k < 0 || k >= b->e->S || !n_out) return DEM_E_INVALID;
  return engine_read_contacts(*b->e, k, true, cap, n_out, pairs, delta_t);
}

dem_status dem_batch_diagnostics(dem_batch *b, double *out) {
  if (!b) return DEM_E_STATE;
  if (!out) return DEM_E_INVALID;
  return engine_diagnostics(*b->e, out);
}

dem_status dem_batch_use_graph(dem_batch *b, int enable) {
  if (!b) return DEM_E_STATE;
  return engine_use_graph(*b->e, enable);
}

dem_status dem_batch_profile(dem_batch *b, int enable) {
  if (!b) return DEM_E_STATE;
  return engine_profile(*b->e, enable);
}

dem_status dem_batch_profile_read(dem_batch *b, double ms[DEM_NUM_PHASES], int64_t *steps) {
  if (!b) return DEM_E_STATE;
  if (!ms || !steps) return DEM_E_INVALID;
  return engine_profile_read(*b->e, ms, steps);
}

dem_status dem_batch_sync(dem_batch *b) {
  if (!b) return DEM_E_STATE;
  return sync_and_check(*b->e);
}

dem_status dem_batch_destroy(dem_batch *b) {
  if (!b) return DEM_E_STATE;
  release(b->e);
  delete b;
  return DEM_OK;
}

}  // extern "C"
