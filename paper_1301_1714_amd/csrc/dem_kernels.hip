// dem_kernels.hip -- HIP kernels of one DEM timestep for gfx950 (wave64).
//
// Steps of Sec. 4.2 and the kernels that run them (every kernel serves all
// systems of an engine at once; per-particle kernels run blocks that never
// straddle two systems, so a block reads its system's constants once):
//   Steps 1-2    k_kick_drift_hash: opening half kick, drift and the cell
//                hash (CM) fused; between two steps of one call k_gather
//                does it instead, for the next step
//   Step 3       k_count / scan / k_scatter / k_canon: counting sort by cell,
//                ties ordered by particle id, so SCM[j] = CM[SCCM[j]] (Eq. 11)
//                holds with one unique order; the paper's bitonic sort is
//                replaced by this O(N) sort (any correct sort of unique keys
//                gives the same permutation)
//   Step 4       k_reorder: gather the state into the sorted order as one
//                packed record per particle, plus an FP32 copy of (x - lo, r)
//                for the detection prefilter
//   Steps 5-8    k_contacts_direct: each particle sweeps the forward half of
//                the 27 cells of Eq. 12, rejects with a conservative
//                fixed-point test and decides the rest exactly in FP64; its
//                contacts (ascending slot order, then its walls) form the
//                list of contacts it owns.  In the same pass each wave then
//                evaluates its particles' contacts one lane per contact
//                (compacted by a prefix sum over the wave, so every lane has a
//                real contact): the law (Eqs. 2-10, or Eq. 1) once per pair,
//                seen from the owner, with the history looked up in the
//                committed table; the result is stored per contact and filed
//                in the partner's backward list.  k_detect_cells /
//                k_detect_tiles build the same lists with other launch
//                shapes; k_contact_law then runs the law pass for them.
//   Steps 7-8    k_gather: one lane per particle sums its contacts in a fixed
//                order (no float atomics) and applies the closing half kick
// No step is a dense contraction, so nothing here uses the matrix cores.
#include <math.h>
#include <string.h>

#include "dem_internal.h"

namespace dem {

__device__ __forceinline__ void raise_err(int32_t *err, int32_t bit) { atomicOr(err, bit); }

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// --------------------------------------------------------------------------
// exact arithmetic shared by detection and hashing: no contraction into FMA,
// so that the result is the one of the plain expression

__device__ __forceinline__ double dist2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ double sq_exact(double s) {
#pragma clang fp contract(off)
  return s * s;
}

// Step 2: global cell of a position (Sec. 4.1).  Returns false when the
// particle is more than one cell outside the box (or not finite).
__device__ __forceinline__ bool hash_cell(const Grid &g, double x, double y, double z, int32_t *cell) {
#pragma clang fp contract(off)
  const double p[3] = {x, y, z};
  int32_t ijk[3];
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    double u = (p[a] - g.lo[a]) * g.sc[a];
    ok = ok && (u >= -1.0 && u < (double)g.nc[a] + 1.0);
    // clamped in floating point before the conversion, so that a position
    // out of range or not a number (an error already flagged) still gives a
    // cell of the grid
    double f = floor(u);
    f = f >= 0.0 ? f : 0.0;
    f = f <= (double)(g.nc[a] - 1) ? f : (double)(g.nc[a] - 1);
    ijk[a] = (int32_t)f;
  }
  *cell = g.c0 + ijk[0] + g.nc[0] * (ijk[1] + g.nc[1] * ijk[2]);
  return ok;
}

// c - q for q the nearest point of plate P to the centre c (the selects of
// the clamp are exact, so the result is the plain expression's)
__device__ __forceinline__ void plate_gap(const Plate &P, const double c[3], double d[3]) {
  const int ax = P.axis, u = ax == 2 ? 0 : ax + 1, v = ax == 0 ? 2 : ax - 1;
  double q[3];
  q[ax] = P.at;
  q[u] = c[u] < P.lo[0] ? P.lo[0] : (c[u] > P.hi[0] ? P.hi[0] : c[u]);
  q[v] = c[v] < P.lo[1] ? P.lo[1] : (c[v] > P.hi[1] ? P.hi[1] : c[v]);
#pragma unroll
  for (int k = 0; k < 3; k++) d[k] = c[k] - q[k];
}

// Step 8: fn(-1 - w) for every wall w the sphere (centre c, radius r)
// touches, in ascending w: the box walls of the mask (w = 0..5: gap < r),
// then the plates (w = 6 + k: nearest-point distance d^2 < r^2)
template <typename Fn>
__device__ __forceinline__ void for_walls(const SysInfo &si, const double c[3], float r, Fn &&fn) {
  const uint32_t wall_mask = si.c.wall_mask;
  const double rid = (double)r;
  if (wall_mask) {
    for (int w = 0; w < 6; w++) {
      if (!((wall_mask >> w) & 1)) continue;
      const int ax = w >> 1;
      const double gap = (w & 1) ? (si.g.hi[ax] - c[ax]) : (c[ax] - si.g.lo[ax]);
      if (gap < rid) fn(-1 - w);
    }
  }
  for (int k = 0; k < si.nplates; k++) {
    double d[3];
    plate_gap(si.plates[k], c, d);
    if (dist2_exact(d[0], d[1], d[2]) < sq_exact(rid)) fn(-7 - k);
  }
}

template <typename Real>
__device__ __forceinline__ Real mass_of(const Consts &c, Real r) {
  return (Real)c.mass_c * r * r * r;
}

// the slot of this thread in a per-particle launch, or -1; k: its system
__device__ __forceinline__ int32_t block_slot(const Layout &L, int32_t &k) {
  k = L.bsys[blockIdx.x];
  const int32_t s = L.bfirst[blockIdx.x] + (int32_t)threadIdx.x;
  const SysInfo &si = L.tab[k];
  return s < si.p0 + si.n ? s : -1;
}

__device__ __forceinline__ bool is_active(const StepCtl &ctl, int32_t k) { return *ctl.step < ctl.left[k]; }

// --------------------------------------------------------------------------
// Steps 1-2

__global__ __launch_bounds__(kBlock) void k_hash(Layout L, PosBuf p, int32_t *cell, int32_t *err) {
  int32_t k;
  const int32_t i = block_slot(L, k);
  if (i < 0) return;
  int32_t c;
  if (!hash_cell(L.tab[k].g, p.x[i], p.y[i], p.z[i], &c)) raise_err(err, ERR_DOMAIN);
  cell[i] = c;
}

template <typename Real>
__device__ __forceinline__ void half_kick(const Consts &c, Real m, Real I, const Real F[3], const Real T[3],
                                          Real v[3], Real w[3]) {
#pragma clang fp contract(off)
  const Real h = (Real)c.half_dt;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    v[k] += h * (F[k] / m + (Real)c.g[k]);
    w[k] += h * (T[k] / I);
  }
}

// Step 1 drift x += dt v and Step 2 hash of the new position
template <typename Real>
__device__ __forceinline__ void drift_hash(const PosBuf &p, int32_t i, const Real v[3], const Consts &c,
                                           const Grid &g, int32_t *cell, int32_t *err) {
#pragma clang fp contract(off)
  const double x = p.x[i] + c.dt * (double)v[0];
  const double y = p.y[i] + c.dt * (double)v[1];
  const double z = p.z[i] + c.dt * (double)v[2];
  p.x[i] = x;
  p.y[i] = y;
  p.z[i] = z;
  int32_t cc;
  if (!hash_cell(g, x, y, z, &cc)) raise_err(err, ERR_DOMAIN);
  cell[i] = cc;
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_kick_drift_hash(Layout L, StepCtl ctl, PosBuf p, VelBuf vb,
                                                            const Real *__restrict__ Fx,
                                                            const Real *__restrict__ Fy,
                                                            const Real *__restrict__ Fz,
                                                            const Real *__restrict__ Tx,
                                                            const Real *__restrict__ Ty,
                                                            const Real *__restrict__ Tz,
                                                            const int32_t *__restrict__ scell, int32_t *cell,
                                                            int32_t *err) {
  int32_t k;
  const int32_t i = block_slot(L, k);
  if (i < 0) return;
  if (!is_active(ctl, k)) {
    cell[i] = scell[i];  // not moving: the next sort sees its current cell
    return;
  }
  const SysInfo &si = L.tab[k];
  Real *V[3] = {(Real *)vb.v[0], (Real *)vb.v[1], (Real *)vb.v[2]};
  Real *Wv[3] = {(Real *)vb.w[0], (Real *)vb.w[1], (Real *)vb.w[2]};
  const Real r = (Real)p.r[i];
  const Real m = mass_of<Real>(si.c, r);
  const Real I = (Real)0.4 * m * r * r;
  Real v[3] = {V[0][i], V[1][i], V[2][i]};
  Real w[3] = {Wv[0][i], Wv[1][i], Wv[2][i]};
  const Real F[3] = {Fx[i], Fy[i], Fz[i]};
  const Real T[3] = {Tx[i], Ty[i], Tz[i]};
  half_kick<Real>(si.c, m, I, F, T, v, w);
#pragma unroll
  for (int q = 0; q < 3; q++) {
    V[q][i] = v[q];
    Wv[q][i] = w[q];
  }
  drift_hash(p, i, v, si.c, si.g, cell, err);
}

// --------------------------------------------------------------------------
// Step 3: counting sort by cell, then a canonical order (by id) inside cells

__global__ __launch_bounds__(kBlock) void k_fill(int32_t *a, int64_t len, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < len) a[i] = value;
}

// Cell counts and each particle's rank in its cell.  The input is in the
// previous step's sorted order, so neighbouring lanes mostly share a cell:
// each run of equal cells within a wave takes one atomic for its length,
// and its ranks follow the input order, which is the cell's id order when
// the cell's particles all stayed in it.  A cell whose order inside still
// has to be set is flagged: one that a particle entered or left, or whose
// particles may have drawn their ranks with more than one atomic (a run at
// either end of a wave); with no previous cells (a first sort), every cell.
__global__ __launch_bounds__(kBlock) void k_count(const int32_t *__restrict__ cell,
                                                  const int32_t *__restrict__ cell_old, int32_t *__restrict__ rank,
                                                  int32_t *counts, uint8_t *flags, int32_t n) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  const int32_t c = valid ? cell[i] : -1;
  const int lane = threadIdx.x & 63;
  const int32_t prev = __shfl_up(c, 1);
  const bool head = !valid || lane == 0 || prev != c;  // invalid lanes end every run
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const int start = 63 - __clzll(heads & upto);
  const unsigned long long above = heads & ~upto;
  const int next = above ? __ffsll((long long)above) - 1 : 64;
  int32_t base = 0;
  if (valid && head) base = atomicAdd(&counts[c], next - lane);
  if (valid && head && (cell_old == nullptr || lane == 0 || next == 64)) flags[c] = 1;
  if (valid && cell_old != nullptr) {
    const int32_t co = cell_old[i];
    if (co != c) {
      flags[c] = 1;
      flags[co] = 1;
    }
  }
  base = __shfl(base, start);
  if (valid) rank[i] = base + (lane - start);
}

constexpr int kScanItems = 16;
constexpr int kScanChunk = kBlock * kScanItems;  // 4096 entries per block

// exclusive scan of one 4096-entry chunk; the chunk total goes to sums[block]
__global__ __launch_bounds__(kBlock) void k_scan_local(const int32_t *in, int32_t *out, int64_t len,
                                                       int32_t *sums) {
  __shared__ int32_t tile[kScanChunk];
  __shared__ int32_t part[kBlock];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  for (int k = 0; k < kScanItems; k++) {
    const int64_t idx = base + k * kBlock + tid;
    tile[k * kBlock + tid] = idx < len ? in[idx] : 0;
  }
  __syncthreads();
  int32_t tot = 0;
  for (int k = 0; k < kScanItems; k++) tot += tile[tid * kScanItems + k];
  part[tid] = tot;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int32_t t = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += t;
    __syncthreads();
  }
  int32_t run = part[tid] - tot;
  for (int k = 0; k < kScanItems; k++) {
    const int32_t v = tile[tid * kScanItems + k];
    tile[tid * kScanItems + k] = run;
    run += v;
  }
  __syncthreads();
  for (int k = 0; k < kScanItems; k++) {
    const int64_t idx = base + k * kBlock + tid;
    if (idx < len) out[idx] = tile[k * kBlock + tid];
  }
  if (tid == kBlock - 1) sums[blockIdx.x] = part[kBlock - 1];
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t *out, int64_t len, const int32_t *offs) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int32_t o = offs[blockIdx.x];
  for (int k = 0; k < kScanItems; k++) {
    const int64_t idx = base + k * kBlock + threadIdx.x;
    if (idx < len) out[idx] += o;
  }
}

// out[len] = out[len-1] + in[len-1]
__global__ void k_scan_total(const int32_t *in, int32_t *out, int64_t len) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[len] = len > 0 ? out[len - 1] + in[len - 1] : 0;
}

static hipError_t scan_exclusive(const int32_t *in, int32_t *out, int64_t len, const ScanScratch &sc, int level,
                                 hipStream_t st) {
  if (len <= 0) return hipSuccess;
  const int64_t nb = (len + kScanChunk - 1) / kScanChunk;
  int32_t *sums = sc.level[level];
  k_scan_local<<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(in, out, len, sums);
  if (nb > 1) {
    hipError_t e = scan_exclusive(sums, sums, nb, sc, level + 1, st);
    if (e != hipSuccess) return e;
    k_scan_add<<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(out, len, sums);
  }
  return hipGetLastError();
}

// exclusive scan with the total in out[len]
static hipError_t scan_with_total(const int32_t *in, int32_t *out, int64_t len, const ScanScratch &sc,
                                  hipStream_t st) {
  hipError_t e = scan_exclusive(in, out, len, sc, 0, st);
  if (e != hipSuccess) return e;
  k_scan_total<<<1, 64, 0, st>>>(in, out, len);
  return hipGetLastError();
}

int64_t scan_scratch_len(int64_t n, int64_t *lens, int *nlevels) {
  int64_t total = 0;
  int l = 0;
  int64_t len = n;
  while (true) {
    const int64_t nb = (len + kScanChunk - 1) / kScanChunk;
    if (l < 4) lens[l] = nb > 0 ? nb : 1;
    total += nb > 0 ? nb : 1;
    l++;
    if (nb <= 1) break;
    len = nb;
  }
  *nlevels = l;
  return total;
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t *__restrict__ cell,
                                                    const int32_t *__restrict__ rank,
                                                    const int32_t *__restrict__ cell_start,
                                                    int32_t *__restrict__ perm, int32_t n) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  perm[cell_start[cell[i]] + rank[i]] = i;
}

// Each flagged cell's slots ordered by particle id (and its flag cleared).
// Cells of up to kCanonSerial particles (the usual handful): one thread.
constexpr int32_t kCanonSerial = 32;
constexpr int32_t kCanonChunk = 4096;  // cells scanned per workgroup by k_canon_big
constexpr int32_t kCanonIds = 1024;    // ids staged in LDS per round of k_canon_big

constexpr int32_t kCanonReg = 8;  // cells up to this size are sorted in registers

__global__ __launch_bounds__(kBlock) void k_canon(const int32_t *__restrict__ cell_start,
                                                  const int32_t *__restrict__ id_old, int32_t *perm,
                                                  uint8_t *flags, int64_t ncell) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell || flags[c] == 0) return;
  flags[c] = 0;
  const int32_t beg = cell_start[c], end = cell_start[c + 1], n = end - beg;
  if (n <= 1 || n > kCanonSerial) return;  // nothing to order, or a crowded cell: k_canon_big
  if (n <= kCanonReg) {
    // the cell's entries and their ids loaded together (two rounds of
    // loads, not one per step of an insertion), ordered by a sorting
    // network (odd-even transposition) in registers
    int32_t P[kCanonReg], I[kCanonReg];
#pragma unroll
    for (int i = 0; i < kCanonReg; i++) P[i] = i < n ? perm[beg + i] : 0;
#pragma unroll
    for (int i = 0; i < kCanonReg; i++) I[i] = i < n ? id_old[P[i]] : INT32_MAX;
#pragma unroll
    for (int r = 0; r < kCanonReg; r++) {
#pragma unroll
      for (int i = r & 1; i + 1 < kCanonReg; i += 2) {
        const bool sw = I[i] > I[i + 1];
        const int32_t a0 = I[i], a1 = I[i + 1], b0 = P[i], b1 = P[i + 1];
        I[i] = sw ? a1 : a0;
        I[i + 1] = sw ? a0 : a1;
        P[i] = sw ? b1 : b0;
        P[i + 1] = sw ? b0 : b1;
      }
    }
#pragma unroll
    for (int i = 0; i < kCanonReg; i++)
      if (i < n) perm[beg + i] = P[i];
    return;
  }
  for (int32_t k = beg + 1; k < end; k++) {
    const int32_t pk = perm[k];
    const int32_t key = id_old[pk];
    int32_t j = k - 1;
    while (j >= beg && id_old[perm[j]] > key) {
      perm[j + 1] = perm[j];
      j--;
    }
    perm[j + 1] = pk;
  }
}

// Crowded cells (more than kCanonSerial particles: a degenerate grid or a
// pile-up), each ordered by one workgroup instead of one thread: a
// particle's place in its cell is the number of the cell's ids below its
// own (ids are unique), counted against the ids staged kCanonIds at a time
// in LDS; the permutation goes through tmp and back.
__global__ __launch_bounds__(kBlock) void k_canon_big(const int32_t *__restrict__ cell_start,
                                                      const int32_t *__restrict__ id_old, int32_t *perm,
                                                      int32_t *tmp, int64_t ncell) {
  __shared__ int32_t big[kCanonChunk];
  __shared__ int32_t ids[kCanonIds];
  __shared__ int32_t nbig;
  const int64_t c_lo = (int64_t)blockIdx.x * kCanonChunk;
  if (threadIdx.x == 0) nbig = 0;
  __syncthreads();
  for (int32_t i = threadIdx.x; i < kCanonChunk && c_lo + i < ncell; i += kBlock)
    if (cell_start[c_lo + i + 1] - cell_start[c_lo + i] > kCanonSerial) big[atomicAdd(&nbig, 1)] = i;
  __syncthreads();
  const int32_t nb = nbig;
  for (int32_t b = 0; b < nb; b++) {
    const int64_t c = c_lo + big[b];
    const int32_t beg = cell_start[c], n = cell_start[c + 1] - beg;
    for (int32_t e0 = 0; e0 < n; e0 += kBlock) {
      const int32_t e = e0 + (int32_t)threadIdx.x;
      const int32_t key = e < n ? id_old[perm[beg + e]] : 0;
      int32_t r = 0;
      for (int32_t f0 = 0; f0 < n; f0 += kCanonIds) {
        const int32_t m = min(kCanonIds, n - f0);
        __syncthreads();
        for (int32_t f = threadIdx.x; f < m; f += kBlock) ids[f] = id_old[perm[beg + f0 + f]];
        __syncthreads();
        for (int32_t f = 0; f < m; f++) r += ids[f] < key ? 1 : 0;
      }
      if (e < n) tmp[beg + r] = perm[beg + e];
    }
    __syncthreads();
    for (int32_t e = threadIdx.x; e < n; e += kBlock) perm[beg + e] = tmp[beg + e];
    __syncthreads();
  }
}

hipError_t launch_sort(const int32_t *cell, const int32_t *id_old, const int32_t *cell_old, int32_t n,
                       int64_t ncell, int32_t *counts, int32_t *rank, int32_t *cell_start, int32_t *perm,
                       uint8_t *flags, const ScanScratch &sc, hipStream_t st) {
  k_fill<<<blocks_for(ncell), kBlock, 0, st>>>(counts, ncell, 0);
  if (n > 0) k_count<<<blocks_for(n), kBlock, 0, st>>>(cell, cell_old, rank, counts, flags, n);
  hipError_t e = scan_with_total(counts, cell_start, ncell, sc, st);
  if (e != hipSuccess) return e;
  if (n > 0) {
    k_scatter<<<blocks_for(n), kBlock, 0, st>>>(cell, rank, cell_start, perm, n);
    k_canon<<<blocks_for(ncell), kBlock, 0, st>>>(cell_start, id_old, perm, flags, ncell);
    // rank is free once scattered: the crowded cells' permutation passes through it
    k_canon_big<<<(unsigned)((ncell + kCanonChunk - 1) / kCanonChunk), kBlock, 0, st>>>(cell_start, id_old, perm,
                                                                                      rank, ncell);
  }
  return hipGetLastError();
}

hipError_t launch_fill(int32_t *a, int64_t len, int32_t value, hipStream_t st) {
  if (len > 0) k_fill<<<blocks_for(len), kBlock, 0, st>>>(a, len, value);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Step 4: gather into the sorted order

__device__ __forceinline__ float4 make_xyzr(const Grid &g, double x, double y, double z, float r) {
  return make_float4((float)(x - g.lo[0]), (float)(y - g.lo[1]), (float)(z - g.lo[2]), r);
}

// The direct sweep's candidate record, 8 bytes instead of the 16 of the FP32
// copy (the sweep is bound by the loads of its candidates).  Every length is
// in one unit h = (widest cell side) / 8192 of the system's grid: each
// coordinate (x - lo) / h rounded to an integer and kept modulo 2^16 (8
// cells of the widest side), the radius r / h rounded up.  The difference of
// two coordinates read as a signed 16-bit number is then the rounded
// difference reduced to [-4, 4) widest cells: exact to one unit where the
// true difference lies in that range, and never larger in magnitude than the
// true one outside it.  A pair in contact is at most one cell_size apart,
// which is at most 2 widest cells (cell divisor <= 2), so its differences
// are exact to one unit on each axis, and an integer test of the squared
// distance against (r_i + r_j + margin)^2 in units of h passes every true
// contact (the wrapped differences of far pairs only make it pass more).
constexpr double kFixCell = 8192.0;
// h^-1 of the system's grid
__device__ __forceinline__ double fix_scale(const Grid &g) {
  return kFixCell * fmin(fmin(g.sc[0], g.sc[1]), g.sc[2]);
}
__device__ __forceinline__ uint32_t fix_coord(double u) {
  double f = floor(u + 0.5);
  // a position far outside the grid or not a number (a step that has failed
  // with the domain error) gets a defined record instead of an out-of-range
  // conversion
  f = fabs(f) < 4.0e15 ? f : 0.0;
  return (uint32_t)(int64_t)f & 0xffffu;
}
__device__ __forceinline__ uint2 make_xq(const SysInfo &si, double x, double y, double z, float r) {
  const Grid &g = si.g;
  const double sc = fix_scale(g);
  const uint32_t qx = fix_coord((x - g.lo[0]) * sc), qy = fix_coord((y - g.lo[1]) * sc),
                 qz = fix_coord((z - g.lo[2]) * sc);
  const double rr = ceil((double)r * sc);
  const uint32_t qr = rr <= 0.0 ? 0u : (rr >= 16383.0 ? 16383u : (uint32_t)rr);
  return make_uint2(qx | (qy << 16), qz | (qr << 16));
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_reorder(Layout L, PosBuf src, VelBuf vsrc, PosBuf dst, VelBuf vdst,
                                                    int32_t soa, const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ cell, int32_t *__restrict__ scell,
                                                    NbrBuf nb, const int32_t *__restrict__ old_cnt,
                                                    const int32_t *__restrict__ old_start) {
  // the block's packed records are staged here and stored as one contiguous
  // run, 16 bytes per lane and instruction (a record per lane would make
  // every store instruction touch a line per lane)
  __shared__ uint4 stage[kBlock * sizeof(PState<Real>) / 16];
  int32_t k;
  const int32_t s = block_slot(L, k);
  const int32_t s0 = L.bfirst[blockIdx.x];
  const SysInfo &si = L.tab[k];
  const int32_t nval = min(kBlock, si.p0 + si.n - s0);  // the block's slots
  if (s >= 0) {
  const int32_t p = perm[s];
  PState<Real> ps;
  ps.x = src.x[p];
  ps.y = src.y[p];
  ps.z = src.z[p];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    ps.v[q] = ((const Real *)vsrc.v[q])[p];
    ps.w[q] = ((const Real *)vsrc.w[q])[p];
  }
  ps.r = src.r[p];
  ps.id = src.id[p] | ((src.mt ? src.mt[p] : 0) << kMtShift);
  ps.hp = 0;
  ps.hq = 0;
  if (old_cnt) {
    const int32_t c = min(max(old_cnt[p], 0), nb.K);  // a slot owns at most K entries
    ps.hp = (uint32_t)p | ((uint32_t)c << kPrevBits);
    ps.hq = old_start[p];
  }
  // the candidate records are formed ahead of every store, so that the
  // system's grid is read with scalar loads (a store may alias it as far as
  // the compiler knows); the FP32 copies are candidates only of the tiled
  // detection shape, written for the systems that use it
  const uint2 xq = make_xq(si, ps.x, ps.y, ps.z, ps.r);
  const float4 xyzr = make_xyzr(si.g, ps.x, ps.y, ps.z, ps.r);
  const int32_t cp = cell[p];
  ((PState<Real> *)stage)[threadIdx.x] = ps;
  if (si.tile > 0) nb.xyzr[s] = xyzr;
  nb.xq[s] = xq;
  scell[s] = cp;
  if (soa) {
    dst.x[s] = ps.x;
    dst.y[s] = ps.y;
    dst.z[s] = ps.z;
    dst.r[s] = ps.r;
    dst.id[s] = ps.id & kIdMask;
    if (dst.mt) dst.mt[s] = ps.id >> kMtShift;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      ((Real *)vdst.v[q])[s] = ps.v[q];
      ((Real *)vdst.w[q])[s] = ps.w[q];
    }
  }
  }
  __syncthreads();
  constexpr int32_t kChunks = sizeof(PState<Real>) / 16;  // 16-byte pieces per record
  uint4 *dst16 = (uint4 *)((PState<Real> *)nb.pst + s0);
  for (int32_t c = (int32_t)threadIdx.x; c < nval * kChunks; c += kBlock) dst16[c] = stage[c];
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_pack(Layout L, PosBuf pos, VelBuf vel, NbrBuf nb) {
  int32_t k;
  const int32_t s = block_slot(L, k);
  if (s < 0) return;
  PState<Real> ps;
  ps.x = pos.x[s];
  ps.y = pos.y[s];
  ps.z = pos.z[s];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    ps.v[q] = ((const Real *)vel.v[q])[s];
    ps.w[q] = ((const Real *)vel.w[q])[s];
  }
  ps.r = pos.r[s];
  ps.id = pos.id[s] | ((pos.mt ? pos.mt[s] : 0) << kMtShift);
  ps.hp = 0;
  ps.hq = 0;
  ((PState<Real> *)nb.pst)[s] = ps;
}

__global__ __launch_bounds__(kBlock) void k_xyzr(Layout L, PosBuf p, NbrBuf nb) {
  int32_t k;
  const int32_t s = block_slot(L, k);
  if (s < 0) return;
  nb.xyzr[s] = make_xyzr(L.tab[k].g, p.x[s], p.y[s], p.z[s], p.r[s]);
  nb.xq[s] = make_xq(L.tab[k], p.x[s], p.y[s], p.z[s], p.r[s]);
}

// --------------------------------------------------------------------------
// Steps 5-6: contact detection over the 27 cells of Eq. 12.
//
// Each pair is tested once, by its lower slot: a particle visits the
// forward half of its 27 cells -- the rest of its own row of cells after
// itself, the next row along y, the three rows of the next plane along z
// (after the sort each row's three cells are one contiguous slot range).  A
// row, or an end cell of a row, whose box lies farther than r_i + r_max from
// the particle is skipped: a conservative bound (margin 2 eps covers the
// FP32 rounding of the coordinates and the cell faces), so it never skips a
// contact.  Candidates pass a conservative FP32 test; the few survivors are
// decided exactly in FP64.  Rows are visited in (z, y) order and cells in x
// order, so the contacts come out in ascending slot order, then the walls.
//
// Three launch shapes build the same lists: the direct one (one lane per
// particle, candidates read through the caches), the wave one (k_detect_cells
// below: one wave per run of cells, candidates in the lanes, particles in
// turn) and the tiled one (one workgroup per run of cells along x stages the
// FP32 copies of the rows it needs in LDS first).  A system's tile_cells
// selects the shape.

constexpr int kTileThreads = 128;
constexpr int kHaloCap = 1024;  // particles staged per tile; a fuller tile reads global memory
constexpr int kSurv = 8;        // LDS survivor slots per lane

// FP64 position and FP32 radius of slot t, from its packed record (the
// same layout for both Real types up to the radius' offset)
struct XR {
  double x, y, z;
  float r;
};
__device__ __forceinline__ XR state_xr(const NbrBuf &nb, bool f64, int32_t t) {
  XR o;
  if (f64) {
    const PState<double> &q = ((const PState<double> *)nb.pst)[t];
    o.x = q.x;
    o.y = q.y;
    o.z = q.z;
    o.r = q.r;
  } else {
    const PState<float> &q = ((const PState<float> *)nb.pst)[t];
    o.x = q.x;
    o.y = q.y;
    o.z = q.z;
    o.r = q.r;
  }
  return o;
}

constexpr int kListStage = 8;  // list entries a lane keeps in LDS until its sweep ends

// entry nf of slot s's list: one of the first kListStage goes to the lane's
// LDS slots (stride kLanes) and is stored with the rest of the list at the
// end of the sweep, so that a wave writes each list column in one store
// rather than one scattered store per contact as it is found
template <int kLanes>
__device__ __forceinline__ void record(const NbrBuf &nb, int32_t N, int32_t kcap, int32_t s, int32_t *lst,
                                       int32_t t, int32_t &nf) {
  if (nf < kListStage)
    lst[nf * kLanes] = t;
  else if (nf < kcap)
    nb.nb[(int64_t)nf * N + s] = t;
  nf++;
}

// exact FP64 decisions (the contact test of Step 7) on the prefilter's
// survivors surv[0 .. ns) (stride kLanes), in order; the records of two
// survivors are requested together, so that a lane waits for one round trip
// per pair of survivors instead of one per survivor
template <int kLanes>
__device__ __forceinline__ void exact_survivors(const NbrBuf &nb, bool f64, int32_t N, int32_t kcap, int32_t s,
                                                float ri, double xi, double yi, double zi, const int32_t *surv,
                                                int32_t ns, int32_t *lst, int32_t &nf) {
  for (int32_t j0 = 0; j0 < ns; j0 += 2) {
    int32_t t[2];
    XR q[2];
#pragma unroll
    for (int u = 0; u < 2; u++) {
      t[u] = surv[min(j0 + u, ns - 1) * kLanes];
      q[u] = state_xr(nb, f64, t[u]);
    }
#pragma unroll
    for (int u = 0; u < 2; u++) {
      if (j0 + u >= ns) break;
      const double ex = q[u].x - xi, ey = q[u].y - yi, ez = q[u].z - zi;
      const double S = (double)ri + (double)q[u].r;
      if (dist2_exact(ex, ey, ez) < sq_exact(S)) record<kLanes>(nb, N, kcap, s, lst, t[u], nf);
    }
  }
}

// The prefilter on FP32 copies (x - lo, y - lo, z - lo, r): a pair passes
// when its FP32 distance is below the sum of the radii plus the margin eps,
// which covers the rounding of the copies and of the test.
struct NearF32 {
  float px, py, pz, pe;  // pe: own radius + eps
  __device__ __forceinline__ bool operator()(const float4 &q) const {
    const float dx = q.x - px, dy = q.y - py, dz = q.z - pz, sf = pe + q.w;
    return dx * dx + dy * dy + dz * dz < sf * sf;
  }
};

// The same test on the fixed-point records (make_xq), in integers: the
// coordinate differences dx, dy, dz and the sum of the radii c = r_j + R in
// units of h, where R is the own radius plus kFixMargin units (the rounding
// of the two records' coordinates moves the distance by at most sqrt(3)
// units, and the radii are rounded up), and the test dx^2 + dy^2 + dz^2 <
// c^2.  The differences of x and y come from one packed 16-bit subtraction,
// their squares from one dot product; z and c from a second subtraction
// against (z, -R).  No product overflows for a pair within reach (|d| <=
// 16385 units, c <= 16386); for others an overflow can only pass the pair.
constexpr int kFixMargin = 3;
typedef short short2_t __attribute__((ext_vector_type(2)));
struct NearInt {
  uint32_t qxy;  // own x | y << 16
  uint32_t qzr;  // own z | (-R) << 16
  __device__ __forceinline__ bool operator()(const uint2 &q) const {
    const short2_t dxy = __builtin_bit_cast(short2_t, q.x) - __builtin_bit_cast(short2_t, qxy);
    const short2_t dzc = __builtin_bit_cast(short2_t, q.y) - __builtin_bit_cast(short2_t, qzr);
    const int32_t dz = dzc.x, c = dzc.y;
    const int32_t d2 = __builtin_amdgcn_sdot2(dxy, dxy, dz * dz, false);
    return d2 < c * c;
  }
};

// One particle's sweep over the forward half of the (2K + 1)^3 cells around
// its own (K = 1: the 27 cells of Eq. 12).  rows(dy, dz, ca, cb, beg, end,
// shift) gives the slot range [beg, end) of cells ca..cb of the row at
// offset (dy, dz) and where their candidate records are (slot t at rows.src[t -
// shift]); false for a row outside the grid; rows.filter gives the
// prefilter on those records.  The rows are visited in
// ascending slot order: the own row, rows dy = 1..K of the own plane, then
// rows dy = -K..K of planes dz = 1..K.  Survivors wait in the lane's LDS
// slots (stride kLanes) so that the rare exact test does not sit inside the
// candidate loop, where one lane taking it would hold the whole wave.  The
// first kListStage contacts stay in the lane's LDS slots lst (stride kLanes)
// and are also stored to the list; returns the number of contacts kept.
template <int kLanes, int K, typename Rows>
__device__ __forceinline__ int32_t sweep_particle(const Rows &rows, const NbrBuf &nb, bool f64, int32_t N,
                                                  int32_t s, const SysInfo &si, int32_t cx, int32_t cy, int32_t cz,
                                                  int32_t *surv, int32_t *lst, int32_t *err) {
  const int32_t kcap = si.kcap;
  const XR me = state_xr(nb, f64, s);
  const float4 p = make_xyzr(si.g, me.x, me.y, me.z, me.r);
  const double xi = me.x, yi = me.y, zi = me.z;
  const float eps = si.eps;
  const int32_t nx = si.g.nc[0];
  const float wx = (float)(1.0 / si.g.sc[0]), wy = (float)(1.0 / si.g.sc[1]), wz = (float)(1.0 / si.g.sc[2]);
  const float cut = p.w + si.rmax + 2.0f * eps, cut2 = cut * cut;
  // distances to the faces of the own cell (0 for a particle outside it)
  const float dxh = fmaxf((float)(cx + 1) * wx - p.x, 0.0f);
  const float dyl = fmaxf(p.y - (float)cy * wy, 0.0f), dyh = fmaxf((float)(cy + 1) * wy - p.y, 0.0f);
  const float dzh = fmaxf((float)(cz + 1) * wz - p.z, 0.0f);
  const float dxl = fmaxf(p.x - (float)cx * wx, 0.0f);
  const auto near = rows.filter(nb, s, si, p, p.w + eps);
  // the slot ranges of the forward rows first, so that their loads overlap;
  // a row, or a cell at either end of a row, whose box lies beyond cut is
  // skipped (the distance to the row or cell i steps away is the distance to
  // the own cell's face plus i - 1 cell widths)
  constexpr int R = 1 + 2 * K + 2 * K * K;
  int32_t beg[R], end[R], shift[R];
  using Rec = typename Rows::Rec;
  constexpr int kU = Rows::kUnroll;
  static_assert(32 % kU == 0, "a chunk's candidates must fill at most the 32 bits of its mask");
#pragma unroll
  for (int h = 0; h < R; h++) {
    const int dyr = h <= K ? h : (h - K - 1) % (2 * K + 1) - K;
    const int dzr = h <= K ? 0 : 1 + (h - K - 1) / (2 * K + 1);
    const float dy = dyr < 0 ? dyl + (float)(-dyr - 1) * wy : (dyr > 0 ? dyh + (float)(dyr - 1) * wy : 0.0f);
    const float dz = dzr > 0 ? dzh + (float)(dzr - 1) * wz : 0.0f;
    const float dyz2 = dy * dy + dz * dz;
    beg[h] = end[h] = shift[h] = 0;
    if (!(dyz2 < cut2)) continue;
    int32_t ca = cx, cb = cx;
#pragma unroll
    for (int i = 1; i <= K; i++) {
      const float dl = dxl + (float)(i - 1) * wx, dh = dxh + (float)(i - 1) * wx;
      ca = (h > 0 && cx - i >= 0 && dl * dl + dyz2 < cut2) ? cx - i : ca;
      cb = (cx + i < nx && dh * dh + dyz2 < cut2) ? cx + i : cb;
    }
    if (!rows(dyr, dzr, ca, cb, beg[h], end[h], shift[h])) beg[h] = end[h] = 0;
  }
  beg[0] = s + 1;  // own row: the slots after the particle
  int32_t nf = 0, ns = 0;
#pragma unroll
  for (int h = 0; h < R; h++) {
    const int32_t e = end[h], sh = shift[h];
    int32_t t = beg[h];
    // chunks of up to 32 candidates: each candidate's test result is
    // shifted into a bit mask (one add with carry, no branch and no store
    // in the loop), while the next kU candidates are in flight (two
    // register sets take turns; the fetch clamps at the chunk's last
    // candidate); the survivors are then taken from the mask in ascending
    // order and parked in the lane's LDS slots, and decided exactly in FP64
    // (global loads) outside the candidate loop
    while (t < e) {
      const int32_t t0 = t, tc = min(e, t0 + 32);
      uint32_t mask = 0;
      auto test = [&](const Rec (&q)[kU]) {
#pragma unroll
        for (int u = 0; u < kU; u++) {
          const bool pass = (t + u < tc) & near(q[u]);
          mask = mask + mask + (pass ? 1u : 0u);
        }
        t += kU;
      };
      Rec qa[kU], qb[kU];
      rows.fetch(qa, t, tc, sh);
      for (;;) {
        rows.fetch(qb, t + kU, tc, sh);
        test(qa);
        if (t >= tc) break;
        rows.fetch(qa, t + kU, tc, sh);
        test(qb);
        if (t >= tc) break;
      }
      const int32_t top = t - t0 - 1;  // candidate t0 + j sits at bit top - j
      while (mask) {
        const int32_t b = 31 - __builtin_clz(mask);
        mask &= ~(1u << b);
        surv[ns * kLanes] = t0 + top - b;
        if (++ns == kSurv) {
          exact_survivors<kLanes>(nb, f64, N, kcap, s, p.w, xi, yi, zi, surv, ns, lst, nf);
          ns = 0;
        }
      }
      t = tc;
    }
  }
  exact_survivors<kLanes>(nb, f64, N, kcap, s, p.w, xi, yi, zi, surv, ns, lst, nf);
  // Step 8: walls, particles of infinite radius, after the pairs
  {
    const double xs[3] = {xi, yi, zi};
    for_walls(si, xs, p.w, [&](int32_t key) { record<kLanes>(nb, N, kcap, s, lst, key, nf); });
  }
  const int32_t nc = nf < kcap ? nf : kcap;
  for (int32_t j = 0; j < nc && j < kListStage; j++) nb.nb[(int64_t)j * N + s] = lst[j * kLanes];
  if (nf > kcap) raise_err(err, ERR_OVERFLOW);
  nb.fcnt[s] = nc;
  return nc;
}

// two consecutive 8-byte records in one 16-byte load (the records are
// 8-byte aligned; the address unit's cost is per lane and instruction, not
// per byte)
__device__ __forceinline__ uint4 load_two(const uint2 *p) {
  typedef uint4 uint4_a8 __attribute__((aligned(8)));
  return *(const uint4_a8 *)p;
}

struct DirectRows {
  using Rec = uint2;
  static constexpr int kUnroll = 8;  // candidates per pipeline stage (even)
  const uint2 *src;                  // [N + 1]: the last record pads the pair loads
  const int32_t *cell_start;
  int32_t c0, nx, ny, nz, cy, cz;
  __device__ __forceinline__ NearInt filter(const NbrBuf &nb, int32_t s, const SysInfo &si, const float4 &,
                                            float) const {
    const uint2 me = src[s];
    NearInt f;
    f.qxy = me.x;
    const uint32_t R = (me.y >> 16) + (uint32_t)kFixMargin;
    f.qzr = (me.y & 0xffffu) | (((0u - R) & 0xffffu) << 16);
    return f;
  }
  // records t .. t + kUnroll - 1 of a range ending at e (past e: copies of
  // slot e - 1 or the pad, which the caller masks)
  __device__ __forceinline__ void fetch(uint2 (&q)[kUnroll], int32_t t, int32_t e, int32_t) const {
#pragma unroll
    for (int u = 0; u < kUnroll; u += 2) {
      const uint4 w = load_two(src + min(t + u, e - 1));
      q[u] = make_uint2(w.x, w.y);
      q[u + 1] = make_uint2(w.z, w.w);
    }
  }
  __device__ __forceinline__ bool operator()(int dy, int dz, int32_t ca, int32_t cb, int32_t &beg, int32_t &end,
                                             int32_t &shift) const {
    const int32_t yy = cy + dy, zz = cz + dz;
    if (yy < 0 || yy >= ny || zz < 0 || zz >= nz) return false;
    const int32_t row = c0 + (zz * ny + yy) * nx;
    beg = cell_start[row + ca];
    end = cell_start[row + cb + 1];
    shift = 0;
    return true;
  }
};

// --------------------------------------------------------------------------
// Wave-per-cell-run detection (wave64 ballot and compaction).  One wave walks
// a run of kRunCells consecutive cells of one row, taking their particles 64
// consecutive slots at a time.  For each particle, uniform across the wave,
// the lanes hold the candidates of its cell's forward half stencil -- its
// own cell and the next one along x, cells x-1..x+1 of the next row and of
// the three rows of the next plane -- as one concatenated slot range, 64 per
// chunk, loaded coalesced once per cell and kept in registers.  The FP32
// prefilter runs with every lane on that one particle; survivors are appended
// in order (ballot + mbcnt) to the wave's queue in LDS and decided exactly in
// FP64 64 at a time, so the contact branch costs one pass per 64 survivors
// rather than holding a wave per survivor.  A particle's survivors enter the
// queue together and in ascending slot order, so its list is exactly the
// one the per-particle sweep makes.

constexpr int kQueue = 128;    // survivor queue entries per wave
constexpr int kCellWaves = 4;  // waves per workgroup

__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The forward half stencil of cell (cx, cy, cz) as five slot ranges in
// ascending order: rb[h] their first slots, pc[h] the running total of their
// lengths (pc[5] = all candidates).  Rows outside the grid are empty.
struct CellRanges {
  int32_t rb[5], pc[6];
};

__device__ __forceinline__ void cell_ranges(const SysInfo &si, const int32_t *cs, int32_t cx, int32_t cy,
                                                 int32_t cz, CellRanges &R) {
  const int32_t nx = si.g.nc[0], ny = si.g.nc[1], nz = si.g.nc[2], c0 = si.g.c0;
  const int32_t xa = cx > 0 ? cx - 1 : 0, xb = cx < nx - 1 ? cx + 1 : nx - 1;
  const int dys[5] = {0, 1, -1, 0, 1}, dzs[5] = {0, 0, 1, 1, 1};
  R.pc[0] = 0;
#pragma unroll
  for (int h = 0; h < 5; h++) {
    const int32_t yy = cy + dys[h], zz = cz + dzs[h];
    int32_t b = 0, e = 0;
    if (yy >= 0 && yy < ny && zz < nz) {
      const int32_t row = c0 + (zz * ny + yy) * nx;
      b = cs[row + (h == 0 ? cx : xa)];
      e = cs[row + xb + 1];
    }
    R.rb[h] = b;
    R.pc[h + 1] = R.pc[h] + (e - b);
  }
}

// slot of candidate c (0 <= c < pc[5]) of the concatenated ranges
__device__ __forceinline__ int32_t cand_slot(const CellRanges &R, int32_t c) {
  int32_t t = R.rb[0] + c;
#pragma unroll
  for (int h = 1; h < 5; h++) t = c >= R.pc[h] ? R.rb[h] + (c - R.pc[h]) : t;
  return t;
}

__global__ __launch_bounds__(kCellWaves * 64) void k_detect_cells(Layout L, StepCtl ctl, int32_t only_active,
                                                                  bool f64, NbrBuf nb,
                                                                  const int32_t *__restrict__ scell,
                                                                  const int32_t *__restrict__ cell_start,
                                                                  int32_t *err) {
  __shared__ int2 queue_all[kCellWaves][kQueue];  // (particle in group, candidate slot)
  __shared__ int32_t cnt_all[kCellWaves][64];     // contacts so far of each particle of the group
  const int32_t wave = uni((int32_t)(threadIdx.x >> 6)), lane = (int32_t)(threadIdx.x & 63);
  const int32_t run = (int32_t)blockIdx.x * kCellWaves + wave;
  if (run >= L.nruns) return;
  const int4 rr = L.runs[run];
  const int32_t k = uni(rr.x);
  if (only_active && !is_active(ctl, k)) return;  // a finished system keeps its lists
  const SysInfo &si = L.tab[k];
  const int32_t nx = si.g.nc[0], ny = si.g.nc[1], c0 = si.g.c0;
  const int32_t row = uni(rr.y), cy = row % ny, cz = row / ny;
  const int32_t s_lo = uni(cell_start[c0 + row * nx + uni(rr.z)]);
  const int32_t s_hi = uni(cell_start[c0 + row * nx + uni(rr.w) + 1]);
  int2 *queue = queue_all[wave];
  int32_t *cnt = cnt_all[wave];
  const int32_t N = L.n;
  const uint2 *xq = nb.xq;
  const uint64_t lt = (1ull << lane) - 1;  // lanes below this one

  for (int32_t g0 = s_lo; g0 < s_hi; g0 += 64) {
    const int32_t gn = min(64, s_hi - g0);
    cnt[lane] = 0;
    int32_t qh = 0, qt = 0;  // queue head and tail (wave-uniform)

    // decide the queue entries [qh, qh + m) exactly and file the contacts
    auto flush = [&](int32_t m) {
      __builtin_amdgcn_wave_barrier();
      const bool act = lane < m;
      const int2 e = queue[(qh + lane) & (kQueue - 1)];
      const int32_t il = act ? e.x : -1, t = e.y;
      bool ok = false;
      if (act) {
        const XR a = state_xr(nb, f64, g0 + il), b = state_xr(nb, f64, t);
        const double S = (double)a.r + (double)b.r;
        ok = dist2_exact(b.x - a.x, b.y - a.y, b.z - a.z) < sq_exact(S);
      }
      const uint64_t mok = __ballot(ok);
      // a particle's entries are one run of lanes; rs: its first lane
      const int32_t prev = __shfl_up(il, 1), next = __shfl_down(il, 1);
      const uint64_t starts = __ballot(act && (lane == 0 || prev != il));
      const uint64_t mine = starts & (lt | (1ull << lane));
      const int32_t rs = mine ? 63 - __clzll(mine) : 0;
      const int32_t before = __popcll(mok & lt & ~((1ull << rs) - 1));
      if (ok) {
        const int32_t pos = cnt[il] + before;
        if (pos < si.kcap) nb.nb[(int64_t)pos * N + g0 + il] = t;
      }
      __builtin_amdgcn_wave_barrier();
      if (act && (lane == m - 1 || next != il)) cnt[il] += before + (ok ? 1 : 0);
      __builtin_amdgcn_wave_barrier();
      qh += m;
    };

    // each lane loads its particle's candidate record, cell and candidate
    // ranges once; the loops below read them with readlane.  The record is
    // kept as the integer prefilter wants it (see NearInt): x | y << 16 and
    // z | (-R) << 16, R the radius plus the rounding margin.
    const int32_t me = g0 + (lane < gn ? lane : 0);
    const uint2 pr = xq[me];
    const uint32_t pqxy = pr.x;
    const uint32_t pqzr = (pr.y & 0xffffu) | (((0u - ((pr.y >> 16) + (uint32_t)kFixMargin)) & 0xffffu) << 16);
    const int32_t mcell = scell[me];
    CellRanges Rl;
    {
      const int32_t cc = mcell - c0;
      cell_ranges(si, cell_start, cc % nx, cy, cz, Rl);
    }
    const uint64_t starts = __ballot(lane < gn && (lane == 0 || __shfl_up(mcell, 1) != mcell));
    auto ranges_of = [&](int32_t l, CellRanges &R) {
#pragma unroll
      for (int h = 0; h < 5; h++) R.rb[h] = __builtin_amdgcn_readlane(Rl.rb[h], l);
#pragma unroll
      for (int h = 0; h < 6; h++) R.pc[h] = __builtin_amdgcn_readlane(Rl.pc[h], l);
    };
    // A cell with 65..96 candidates tests its second chunk for two
    // particles at once, 32 lanes each: both halves hold candidates 64..95.
    auto halves = [](int32_t C) { return C > 64 && C <= 96; };
    auto load_chunks = [&](const CellRanges &R, uint2 &qa, int32_t &ta, uint2 &qb, int32_t &tb) {
      const int32_t C = R.pc[5];
      const int32_t cb = 64 + (halves(C) ? (lane & 31) : lane);
      ta = lane < C ? cand_slot(R, lane) : -1;
      tb = cb < C ? cand_slot(R, cb) : -1;
      qa = xq[ta >= 0 ? ta : me];
      qb = xq[tb >= 0 ? tb : me];
    };
    // queue the lanes of m (this lane if mine) as contacts of particle l
    auto append = [&](uint64_t m, bool mine, int32_t l, int32_t t) {
      if (!m) return;
      if (mine) {
        const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)qt));
        queue[pos & (kQueue - 1)] = make_int2(l, t);
      }
      qt += __popcll(m);
      if (qt - qh >= 64) flush(64);
    };
    CellRanges R;
    ranges_of(0, R);
    uint2 q0, q1;
    int32_t t0, t1;
    load_chunks(R, q0, t0, q1, t1);
    int32_t a = 0;  // first lane of the current cell
    while (a < gn) {
      // the next cell's first lane and its chunks, in flight while this
      // cell is tested
      const uint64_t later = starts & ~((2ull << a) - 1);
      const int32_t b = later ? __ffsll((long long)later) - 1 : gn;
      CellRanges Rn = R;
      uint2 n0 = q0, n1 = q1;
      int32_t u0 = t0, u1 = t1;
      if (b < gn) {
        ranges_of(b, Rn);
        load_chunks(Rn, n0, u0, n1, u1);
      }
      const int32_t C = R.pc[5];
      const bool split = halves(C);
      for (int32_t l = a; l < b;) {
        const int32_t i = g0 + l;
        const NearInt near_l{(uint32_t)__builtin_amdgcn_readlane((int32_t)pqxy, l),
                             (uint32_t)__builtin_amdgcn_readlane((int32_t)pqzr, l)};
        auto passes = [&](const uint2 &q, int32_t t, const NearInt &near, int32_t ii) {
          return (t > ii) & near(q);
        };
        // chunk 0 of particle l
        {
          const bool ps = passes(q0, t0, near_l, i);
          append(__builtin_amdgcn_ballot_w64(ps), ps, l, t0);
        }
        if (split && l + 1 < b) {
          // chunk 1 of particles l (lanes 0-31) and l + 1 (lanes 32-63);
          // l + 1 files its chunk-1 survivors after its chunk-0 ones
          const NearInt near_n{(uint32_t)__builtin_amdgcn_readlane((int32_t)pqxy, l + 1),
                               (uint32_t)__builtin_amdgcn_readlane((int32_t)pqzr, l + 1)};
          const bool lo = lane < 32;
          const bool p1 = passes(q1, t1, lo ? near_l : near_n, lo ? i : i + 1);
          const uint64_t m1 = __builtin_amdgcn_ballot_w64(p1);
          append(m1 & 0xFFFFFFFFull, p1 && lo, l, t1);
          const bool p0 = passes(q0, t0, near_n, i + 1);
          append(__builtin_amdgcn_ballot_w64(p0), p0, l + 1, t0);
          append(m1 & ~0xFFFFFFFFull, p1 && !lo, l + 1, t1);
          l += 2;
          continue;
        }
        if (C > 64) {
          const bool ps = (!split || lane < 32) && passes(q1, t1, near_l, i);
          append(__builtin_amdgcn_ballot_w64(ps), ps, l, t1);
        }
        for (int32_t cb = 128; cb < C; cb += 64) {  // a crowded stencil: further chunks from the caches
          const int32_t t = cb + lane < C ? cand_slot(R, cb + lane) : -1;
          const bool ps = passes(xq[t >= 0 ? t : me], t, near_l, i);
          append(__builtin_amdgcn_ballot_w64(ps), ps, l, t);
        }
        l += 1;
      }
      R = Rn;
      q0 = n0;
      q1 = n1;
      t0 = u0;
      t1 = u1;
      a = b;
    }
    if (qt > qh) flush(qt - qh);
    // Step 8: walls, particles of infinite radius, after the pairs
    if (lane < gn) {
      const int32_t s = g0 + lane;
      int32_t nf = cnt[lane];
      if (si.c.wall_mask || si.nplates) {
        const XR a = state_xr(nb, f64, s);
        const double xs[3] = {a.x, a.y, a.z};
        for_walls(si, xs, a.r, [&](int32_t key) {
          if (nf < si.kcap) nb.nb[(int64_t)nf * N + s] = key;
          nf++;
        });
      }
      if (nf > si.kcap) raise_err(err, ERR_OVERFLOW);
      nb.fcnt[s] = nf < si.kcap ? nf : si.kcap;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <bool kStaged>
struct TileRows {
  using Rec = float4;
  static constexpr int kUnroll = 2;  // candidates per pipeline stage
  const float4 *src;
  const int32_t (*cs)[kMaxTile + 3];
  int32_t xa;
  int32_t shift[9];
  __device__ __forceinline__ bool operator()(int dy, int dz, int32_t ca, int32_t cb, int32_t &beg, int32_t &end,
                                             int32_t &sh) const {
    const int r = 3 * (dz + 1) + dy + 1;
    beg = cs[r][ca - xa];  // rows outside the grid hold empty ranges
    end = cs[r][cb - xa + 1];
    sh = kStaged ? shift[r] : 0;
    return true;
  }
  __device__ __forceinline__ NearF32 filter(const NbrBuf &, int32_t, const SysInfo &, const float4 &p,
                                            float pe) const {
    return NearF32{p.x, p.y, p.z, pe};
  }
  __device__ __forceinline__ void fetch(float4 (&q)[kUnroll], int32_t t, int32_t e, int32_t sh) const {
#pragma unroll
    for (int u = 0; u < kUnroll; u++) q[u] = src[(uint32_t)(min(t + u, e - 1) - sh)];
  }
};

__global__ __launch_bounds__(kTileThreads) void k_detect_tiles(Layout L, StepCtl ctl, int32_t only_active,
                                                               bool f64, NbrBuf nb,
                                                               const int32_t *__restrict__ scell,
                                                               const int32_t *__restrict__ cell_start,
                                                               int32_t *err) {
  __shared__ float4 halo[kHaloCap];
  __shared__ int32_t cs[9][kMaxTile + 3];  // cell starts of cells xa .. xb + 1 of each row
  __shared__ int32_t surv_all[kSurv * kTileThreads];
  __shared__ int32_t lst_all[kListStage * kTileThreads];
  const int tid = threadIdx.x;
  const int4 tile = L.tiles[blockIdx.x];
  const int32_t k = tile.x;
  if (only_active && !is_active(ctl, k)) return;  // a finished system keeps its lists
  const SysInfo &si = L.tab[k];
  const int32_t nx = si.g.nc[0], ny = si.g.nc[1], nz = si.g.nc[2];
  const int32_t c0 = si.g.c0;
  const int32_t ry = tile.y % ny, rz = tile.y / ny;
  const int32_t x0 = tile.z, x1 = tile.w;
  const int32_t xa = x0 > 0 ? x0 - 1 : 0, xb = x1 < nx - 1 ? x1 + 1 : nx - 1;
  const int32_t wcs = xb - xa + 2;  // cell starts per row
  // the own row and the 4 forward rows (rows 0-3 are not needed: empty)
  for (int32_t i = tid; i < 9 * wcs; i += kTileThreads) {
    const int32_t r = i / wcs, j = i - r * wcs;
    const int32_t yy = ry + (r % 3) - 1, zz = rz + (r / 3) - 1;
    const bool in = r >= 4 && yy >= 0 && yy < ny && zz >= 0 && zz < nz;
    cs[r][j] = in ? cell_start[c0 + (zz * ny + yy) * nx + xa + j] : 0;
  }
  __syncthreads();
  const int32_t own_lo = cs[4][x0 - xa], own_hi = cs[4][x1 - xa + 1];
  if (own_lo == own_hi) return;
  TileRows<true> st;
  st.src = halo;
  st.cs = cs;
  st.xa = xa;
  int32_t total = 0;
#pragma unroll
  for (int r = 0; r < 9; r++) {
    st.shift[r] = cs[r][0] - total;  // slot t of row r sits at halo[t - shift[r]]
    total += cs[r][wcs - 1] - cs[r][0];
  }
  const bool staged = total <= kHaloCap;  // the same for every thread
  if (staged) {
#pragma unroll
    for (int r = 4; r < 9; r++) {
      const int32_t lo = cs[r][0], len = cs[r][wcs - 1] - lo;
      for (int32_t i = tid; i < len; i += kTileThreads) halo[lo - st.shift[r] + i] = nb.xyzr[lo + i];
    }
  }
  __syncthreads();
  int32_t *surv = surv_all + tid, *lst = lst_all + tid;
  if (staged) {
    for (int32_t s = own_lo + tid; s < own_hi; s += kTileThreads)
      sweep_particle<kTileThreads, 1>(st, nb, f64, L.n, s, si, (scell[s] - c0) % nx, ry, rz, surv, lst, err);
  } else {
    TileRows<false> gr;
    gr.src = nb.xyzr;
    gr.cs = cs;
    gr.xa = xa;
    for (int32_t s = own_lo + tid; s < own_hi; s += kTileThreads)
      sweep_particle<kTileThreads, 1>(gr, nb, f64, L.n, s, si, (scell[s] - c0) % nx, ry, rz, surv, lst, err);
  }
}

// history entry: delta_t in x, y, z and the key's bits in w
__device__ __forceinline__ float key_bits(int32_t key, float) { return __int_as_float(key); }
__device__ __forceinline__ double key_bits(int32_t key, double) { return __longlong_as_double((long long)key); }
__device__ __forceinline__ int32_t entry_key(float w) { return __float_as_int(w); }
__device__ __forceinline__ int32_t entry_key(double w) { return (int32_t)__double_as_longlong(w); }

template <typename Real>
struct Vec4T;
template <>
struct Vec4T<float> {
  using type = float4;
};
template <>
struct Vec4T<double> {
  using type = double4;
};

template <typename Real>
struct Vec2T;
template <>
struct Vec2T<float> {
  using type = float2;
};
template <>
struct Vec2T<double> {
  using type = double2;
};

// per-contact record of the law: force on the owner and n x F_t, six Reals
// in three pairs
template <typename Real>
__device__ __forceinline__ void put_record(void *pf, int64_t q, const Real f[3], const Real m[3]) {
  using V2 = typename Vec2T<Real>::type;
  V2 *p = (V2 *)pf + 3 * q;
  V2 a, b, c;
  a.x = f[0];
  a.y = f[1];
  b.x = f[2];
  b.y = m[0];
  c.x = m[1];
  c.y = m[2];
  p[0] = a;
  p[1] = b;
  p[2] = c;
}

template <typename Real>
__device__ __forceinline__ void get_record(const void *pf, int64_t q, Real f[3], Real m[3]) {
  using V2 = typename Vec2T<Real>::type;
  const V2 *p = (const V2 *)pf + 3 * q;
  const V2 a = p[0], b = p[1], c = p[2];
  f[0] = a.x;
  f[1] = a.y;
  f[2] = b.x;
  m[0] = b.y;
  m[1] = c.x;
  m[2] = c.y;
}

template <typename Real>
__device__ __forceinline__ void put_entry(const HistGen &g, int64_t q, const Real d[3], int32_t key) {
  using V4 = typename Vec4T<Real>::type;
  V4 e;
  e.x = d[0];
  e.y = d[1];
  e.z = d[2];
  e.w = key_bits(key, (Real)0);
  ((V4 *)g.ent)[q] = e;
}

// fixed-size bitonic network on registers (indices are compile-time)
// --------------------------------------------------------------------------
// Steps 7-8: contact law

template <typename Real>
struct LawOut {
  Real F[3];     // force on the first body
  Real Ft[3];    // its tangential part (sets the torque of Eq. 3)
  Real dtn[3];   // new tangential displacement (Eq. 7, after Eq. 5)
  Real kn, kt;   // stiffness used (elastic-energy diagnostic)
  Real fn;       // |F_n| of Eq. 4 (0 for the simple law)
};

// One contact seen from body a: n (unit, a -> partner), overlap delta,
// effective radius R and mass M, relative velocity v = v_a - v_b, spin term
// r_a w_a + r_b w_b, previous tangential displacement h; K: the constants of
// the pair's materials.
template <typename Real, int LAW>
__device__ __forceinline__ void contact_law(const Consts &c, const PairK &K, const Real n[3], Real delta, Real R,
                                            Real M, const Real v[3], const Real spin[3], const Real h[3],
                                            LawOut<Real> &o) {
  const Real vn_s = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  const Real sxn[3] = {spin[1] * n[2] - spin[2] * n[1], spin[2] * n[0] - spin[0] * n[2],
                       spin[0] * n[1] - spin[1] * n[0]};
  Real vn[3], vt[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    vn[k] = vn_s * n[k];
    vt[k] = v[k] - vn[k] + sxn[k];  // Eq. 6
  }
  if (LAW == DEM_LAW_SIMPLE) {  // Eq. 1 without gravity
    // the t of Eq. 1 is the tangential component of v (Sec. 3); the simple
    // model has no rotation, so Eq. 6's spin term is not part of it
#pragma unroll
    for (int k = 0; k < 3; k++) {
      o.F[k] = -(Real)c.k_sp * delta * n[k] - (Real)c.k_da * v[k] - (Real)c.k_sh * (v[k] - vn[k]);
      o.Ft[k] = 0;
      o.dtn[k] = 0;
    }
    o.kn = (Real)c.k_sp;
    o.kt = 0;
    o.fn = 0;
    return;
  }
  Real kn, kt;
  if (LAW == DEM_LAW_HERTZ) {  // Eqs. 8-9
    const Real q = sqrt(delta * R);
    kn = (Real)K.kn * q;
    kt = (Real)K.kt * q;
  } else {
    kn = (Real)K.kn;
    kt = (Real)K.kt;
  }
  const Real eta = (Real)K.alpha * sqrt(kn * M);  // Eq. 10
  const Real eta_t = (Real)c.eta_t_ratio * eta;
  const Real hn = h[0] * n[0] + h[1] * n[1] + h[2] * n[2];
  const Real dtc = (Real)c.dt;
  Real Fn[3], Ft[3], dtn[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    dtn[k] = h[k] - hn * n[k] + vt[k] * dtc;  // Eq. 7
    Fn[k] = -kn * delta * n[k] - eta * vn[k];  // Eq. 4
    Ft[k] = -kt * dtn[k] - eta_t * vt[k];
  }
  const Real ftn = sqrt(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
  const Real fnn = sqrt(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2]);
  const Real lim = (Real)K.mu * fnn;
  const bool slip = ftn > lim;  // Eq. 5, evaluated without a branch
  const Real scale = slip ? lim / ftn : (Real)1;
  const bool rescale = slip && kt > (Real)0;
  const Real inv_kt = kt > (Real)0 ? (Real)1 / kt : (Real)0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    Ft[k] *= scale;
    o.dtn[k] = rescale ? -(Ft[k] + eta_t * vt[k]) * inv_kt : dtn[k];
    o.Ft[k] = Ft[k];
    o.F[k] = Fn[k] + Ft[k];  // Eq. 2
  }
  o.kn = kn;
  o.kt = kt;
  o.fn = fnn;
}

// The optional contact terms, each added after the law on its own, so that a
// term is added or removed here without touching the law, the grid or the
// sums: cohesion, a constant pull f_c along n while the bodies overlap;
// rolling resistance, the couple C = -mu_r R |F_n| w_rel / |w_rel| on the
// owner (zero when w_rel = 0) and -C on the partner (the gather applies it).
template <typename Real>
__device__ __forceinline__ void extra_terms(const Consts &c, const Real n[3], Real R, const Real wrel[3],
                                            LawOut<Real> &o, Real C[3]) {
  C[0] = C[1] = C[2] = 0;
  if (c.terms & DEM_TERM_COHESION) {
#pragma unroll
    for (int k = 0; k < 3; k++) o.F[k] += (Real)c.cohesion * n[k];
  }
  if (c.terms & DEM_TERM_ROLLING) {
    const Real wn = sqrt(wrel[0] * wrel[0] + wrel[1] * wrel[1] + wrel[2] * wrel[2]);
    if (wn > (Real)0) {
#pragma unroll
      for (int k = 0; k < 3; k++) C[k] = -(Real)c.rolling_mu * R * o.fn * wrel[k] / wn;
    }
  }
}

template <typename Real, int LAW>
__device__ __forceinline__ double elastic_energy(const Consts &c, const PairK &K, Real delta, Real R,
                                                 const LawOut<Real> &o, const Real h[3]) {
  const double d = (double)delta;
  const double hh = (double)h[0] * h[0] + (double)h[1] * h[1] + (double)h[2] * h[2];
  if (LAW == DEM_LAW_SIMPLE) return 0.5 * c.k_sp * d * d;
  if (LAW == DEM_LAW_HERTZ) return 0.4 * K.kn * sqrt((double)R) * pow(d, 2.5) + 0.5 * (double)o.kt * hh;
  return 0.5 * (double)o.kn * d * d + 0.5 * (double)o.kt * hh;
}

// committed tangential displacement of the contact with history key `key`
// among the c entries from index q0 of the committed table (zero for a new
// contact)
// committed entries of a slot requested together
constexpr int kHistBatch = 4;

template <typename Real>
__device__ __forceinline__ void hist_find(const HistGen &old, int32_t q0, int32_t c, int32_t key, Real h[3]) {
  using V4 = typename Vec4T<Real>::type;
  h[0] = h[1] = h[2] = 0;
  // the entries are adjacent: up to four are requested together, then
  // matched (a lookup waits for one round trip instead of one per entry)
  constexpr int kBatch = kHistBatch;
  for (int32_t k0 = 0; k0 < c; k0 += kBatch) {
    V4 d[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; j++)
      if (k0 + j < c) d[j] = ((const V4 *)old.ent)[(int64_t)q0 + k0 + j];
    bool found = false;
#pragma unroll
    for (int j = 0; j < kBatch; j++) {
      if (!found && k0 + j < c && entry_key(d[j].w) == key) {
        h[0] = d[j].x;
        h[1] = d[j].y;
        h[2] = d[j].z;
        found = true;
      }
    }
    if (found) break;
  }
}

// where a slot's committed history is: its previous slot, the number of its
// entries and the index of the first
struct HistAt {
  int32_t prev, cnt, q0;
};

// where the committed history of slot s (packed record ps) is: recorded in
// the record in a time step, the slot's own otherwise
template <typename Real>
__device__ __forceinline__ HistAt hist_index(const PairArgs &a, bool old_perm, int32_t s, const PState<Real> &ps) {
  if (old_perm) return HistAt{(int32_t)(ps.hp & ((1u << kPrevBits) - 1)), (int32_t)(ps.hp >> kPrevBits), ps.hq};
  return HistAt{s, min(max(a.old.cnt[s], 0), a.nb.K), a.old.start[s]};
}

// a lane's own particle's committed history location (passed to the lanes
// of its contacts; none for the simple law or a lane without a particle)
template <typename Real, int LAW>
__device__ __forceinline__ HistAt owner_history(const PairArgs &a, int32_t s) {
  if ((LAW & 3) == DEM_LAW_SIMPLE || s < 0) return HistAt{0, 0, 0};
  const bool old_perm = (a.mode & MODE_OLD_PERM) != 0;
  if (old_perm) {
    const PState<Real> &ps = ((const PState<Real> *)a.nb.pst)[s];
    return HistAt{(int32_t)(ps.hp & ((1u << kPrevBits) - 1)), (int32_t)(ps.hp >> kPrevBits), ps.hq};
  }
  return HistAt{s, min(max(a.old.cnt[s], 0), a.nb.K), a.old.start[s]};
}

// Owned contact kr of slot s (partner t, a slot or -1 - w), stored at index
// q of the per-contact arrays: the law of Eqs. 2-10 (or Eq. 1) evaluated
// once per pair, seen from the owner (the lower slot), stored as the force
// on the owner and n x F_t; the partner receives the exact negation (its
// sums find the contact where it is filed, back[filed], or in the owner's
// list).  Both particles' inputs come from their packed state records; hs
// says where the owner's committed history is.
template <typename Real, int LAW>
__device__ __forceinline__ void contact_one(const PairArgs &a, const SysInfo &si, int32_t s, int32_t t, int32_t q,
                                            int64_t filed, const HistAt &hs, int32_t kr) {
  constexpr int BASE = LAW & 3;                       // the dem_law
  constexpr bool TERMS = (LAW & kLawTerms) != 0;      // optional terms compiled in
  constexpr bool FULL = (LAW & kLawFull) != 0;        // material tables and diagnostics compiled in
  const PState<Real> *PS = (const PState<Real> *)a.nb.pst;
  const bool old_perm = (a.mode & MODE_OLD_PERM) != 0;
  const bool write_hist = (a.mode & MODE_WRITE_HIST) != 0 && BASE != DEM_LAW_SIMPLE;
  const bool diag = FULL && (a.mode & MODE_DIAG) != 0;
  const Consts &c = si.c;
  // the owner's committed entry at the contact's own rank kr in the
  // owner's list is requested with the records (the owner's lane passed
  // where the owner's entries are): the previous step filed the contact
  // there unless the pair's order changed or a contact before it came or
  // went, in which case the owner's or the partner's entries are searched
  using V4 = typename Vec4T<Real>::type;
  V4 pre;
  if (BASE != DEM_LAW_SIMPLE && hs.cnt > 0) pre = ((const V4 *)a.old.ent)[(int64_t)hs.q0 + min(kr, hs.cnt - 1)];
  const PState<Real> me = PS[s];
  const PState<Real> pt = PS[t >= 0 ? t : s];  // a wall reads the owner twice
  // where the partner side's sums find the contact (the place was drawn by
  // an atomic whose round trip the loads above overlap; stored before the
  // law so that the place and the index need no registers during it)
  if (filed >= 0) a.w.back[filed] = make_int2(q, t);
  Real h[3] = {0, 0, 0};
  if (BASE != DEM_LAW_SIMPLE) {
    if (t >= 0) {
      const HistAt hp = hist_index(a, old_perm, t, pt);
      if (hs.prev < hp.prev) {  // the owner was the lower slot then too
        if (hs.cnt > 0 && entry_key(pre.w) == hp.prev) {
          h[0] = pre.x;
          h[1] = pre.y;
          h[2] = pre.z;
        } else {
          hist_find<Real>(a.old, hs.q0, hs.cnt, hp.prev, h);
        }
      } else {
        hist_find<Real>(a.old, hp.q0, hp.cnt, hs.prev, h);
        h[0] = -h[0];
        h[1] = -h[1];
        h[2] = -h[2];
      }
    } else {
      if (hs.cnt > 0 && entry_key(pre.w) == t) {
        h[0] = pre.x;
        h[1] = pre.y;
        h[2] = pre.z;
      } else {
        hist_find<Real>(a.old, hs.q0, hs.cnt, t, h);
      }
    }
  }
  // the constants of the pair's materials (a wall is of the system's wall
  // material), or the system's one material
  PairK K{c.kn, c.kt, c.alpha, c.mu};
  if (FULL && si.ntypes > 0)
    K = a.L.mat[si.mat0 + (me.id >> kMtShift) * si.ntypes + (t >= 0 ? (pt.id >> kMtShift) : si.wall_type)];
  const float rsf = me.r;
  const Real rs = (Real)rsf;
  const Real ms = mass_of<Real>(c, rs);
  LawOut<Real> o;
  Real n[3], delta, R;
  if (t >= 0) {
    const double dx = pt.x - me.x, dy = pt.y - me.y, dz = pt.z - me.z;
    const double d2 = dist2_exact(dx, dy, dz);
    const double S = (double)rsf + (double)pt.r;
    const Real rt = (Real)pt.r;
    const Real mt = mass_of<Real>(c, rt);
    const Real dd = sqrt((Real)d2);
    const Real invd = (Real)1 / dd;
    n[0] = (Real)dx * invd;
    n[1] = (Real)dy * invd;
    n[2] = (Real)dz * invd;
    delta = (Real)(sq_exact(S) - d2) / ((Real)S + dd);
    R = rs * rt / (rs + rt);
    const Real M = ms * mt / (ms + mt);
    Real v[3], spin[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      v[i] = me.v[i] - pt.v[i];
      spin[i] = rs * me.w[i] + rt * pt.w[i];
    }
    contact_law<Real, BASE>(c, K, n, delta, R, M, v, spin, h, o);
  } else {
    // Step 8: wall -1 - t, a particle of infinite radius: a box wall, or
    // a plate touched at its nearest point
    const int w = -1 - t;
    const double xw[3] = {me.x, me.y, me.z};
    if (w >= 6) {
      double d[3];
      plate_gap(si.plates[w - 6], xw, d);
      const double d2 = dist2_exact(d[0], d[1], d[2]);
      const double dist = sqrt(d2);
#pragma unroll
      for (int i = 0; i < 3; i++) n[i] = (Real)(-d[i] / dist);
      // r - d from r^2 - d^2 (as for pairs): a resting sphere's overlap is
      // many orders below r, and this form does not carry the rounding of
      // the square root into it
      delta = (Real)((sq_exact((double)rsf) - d2) / ((double)rsf + dist));
    } else {
      const int ax = w >> 1;
      const double gap = (w & 1) ? (si.g.hi[ax] - xw[ax]) : (xw[ax] - si.g.lo[ax]);
      n[0] = n[1] = n[2] = 0;
      n[ax] = (w & 1) ? (Real)1 : (Real)-1;
      delta = (Real)((double)rsf - gap);
    }
    R = rs;
    Real spin[3];
#pragma unroll
    for (int i = 0; i < 3; i++) spin[i] = rs * me.w[i];
    contact_law<Real, BASE>(c, K, n, delta, rs, ms, me.v, spin, h, o);
  }
  if (TERMS) {
    Real wrel[3], C[3];
#pragma unroll
    for (int i = 0; i < 3; i++) wrel[i] = t >= 0 ? me.w[i] - pt.w[i] : me.w[i];
    extra_terms<Real>(c, n, R, wrel, o, C);
    using V4 = typename Vec4T<Real>::type;
    V4 cv;
    cv.x = C[0];
    cv.y = C[1];
    cv.z = C[2];
    cv.w = 0;
    ((V4 *)a.w.pc)[q] = cv;
  }
  const Real tq[3] = {n[1] * o.Ft[2] - n[2] * o.Ft[1], n[2] * o.Ft[0] - n[0] * o.Ft[2],
                      n[0] * o.Ft[1] - n[1] * o.Ft[0]};
  put_record<Real>(a.w.pf, q, o.F, tq);
  if (write_hist) put_entry<Real>(a.cur, q, o.dtn, t);
  if (diag) {
    a.w.pe[q] = elastic_energy<Real, BASE>(c, K, delta, R, o, h);
    a.w.pd[q] = (double)delta;
  }
}

// The owned contacts of one wave's particles (lane l: slot first + l, cnt
// contacts), one lane per contact in owner order, 64 at a time, so that
// every lane of the wave evaluates a real contact however unevenly the
// contacts fall on the particles (the contact-branch divergence of a lane per
// particle).  Contact k of lane l is read from lst[k * stride + l] for k <
// kListStage when lst is given (the detection's LDS copy), else from the
// list in global memory.  The wave's contacts are stored from index qbase
// on, in that order.  woff: 65 ints of LDS for the wave.  Every lane of the
// wave must call it.
template <typename Real, int LAW>
__device__ __forceinline__ void law_wave(const PairArgs &a, const SysInfo &si, int32_t first, int32_t cnt,
                                         const int32_t *lst, int32_t stride, int32_t *woff, int32_t qbase,
                                         const HistAt &own) {
  const int32_t lane = (int32_t)(threadIdx.x & 63);
  int32_t x = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  const int32_t total = __shfl(x, 63);
  woff[lane] = x - cnt;
  if (lane == 63) woff[64] = total;
  __builtin_amdgcn_wave_barrier();
  const int32_t s0 = a.L.bfirst[blockIdx.x];
  for (int32_t e0 = 0; e0 < total; e0 += 64) {
    const int32_t e = e0 + lane;
    int32_t k = 0, s = 0, t = -1, tb = -1, lo = 0;
    if (e < total) {
      int32_t hi = 64;  // woff[lo] <= e < woff[hi]
      while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (woff[mid] <= e)
          lo = mid;
        else
          hi = mid;
      }
      k = e - woff[lo];
      s = first + lo;
      t = (lst && k < kListStage) ? lst[k * stride + lo] : a.nb.nb[(int64_t)k * a.L.n + s];
      // the kernel block whose slots the partner is one of
      if (t >= 0) tb = (int32_t)blockIdx.x + ((t - s0) >> 8);
    }
    // the chunk's contacts filed with their partners' blocks: lanes of one
    // block form a group, whose first lane draws the group's places with
    // one atomic
    uint64_t todo = __ballot(tb >= 0);
    int32_t lead = 0, rank = 0, size = 0;
    while (todo) {
      const int32_t l = __builtin_ctzll(todo);
      const int32_t b = __builtin_amdgcn_readlane(tb, l);
      const uint64_t grp = __ballot(tb == b);
      if (tb == b) {
        lead = l;
        rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(grp >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)grp, 0u));
        size = __popcll(grp);
      }
      todo &= ~grp;
    }
    int32_t base = 0;
    if (tb >= 0 && rank == 0) base = atomicAdd(&a.w.nback[tb], size);
    base = __shfl(base, lead) + rank;
    // the owner's committed history location, from the owner's lane
    const HistAt ho{__shfl(own.prev, lo), __shfl(own.cnt, lo), __shfl(own.q0, lo)};
    if (e < total) {
      const int64_t filed = tb >= 0 && base < kBackCap ? (int64_t)tb * kBackCap + base : -1;
      contact_one<Real, LAW>(a, si, s, t, qbase + e, filed, ho, k);
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// A system that has finished its steps in this call: its state does not
// move (so its slots do not change) and its committed history is carried
// into the generation being written.
template <typename Real>
__device__ __forceinline__ void carry_history(const PairArgs &a, int32_t s) {
  using V4 = typename Vec4T<Real>::type;
  if (s < 0 || (a.mode & MODE_WRITE_HIST) == 0) return;
  const int32_t c = min(max(a.old.cnt[s], 0), a.nb.K);
  const int32_t q0 = a.old.start[s];
  a.cur.cnt[s] = c;
  a.cur.start[s] = q0;
  for (int32_t k = 0; k < c; k++) ((V4 *)a.cur.ent)[(int64_t)q0 + k] = ((const V4 *)a.old.ent)[(int64_t)q0 + k];
}

// count and first entry of the history generation being written: the owned
// contacts (none for the simple law, which keeps no history)
template <int LAW>
__device__ __forceinline__ void set_hist_count(const PairArgs &a, int32_t s, int32_t cnt, int32_t q0) {
  if (s >= 0 && (a.mode & MODE_WRITE_HIST) != 0) {
    a.cur.cnt[s] = (LAW & 3) == DEM_LAW_SIMPLE ? 0 : cnt;
    a.cur.start[s] = q0;
  }
}

// exclusive prefix sum of c over the block (and its total); every thread
// of the block must call it
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t c, int32_t *wsum, int32_t &total) {
  const int32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t x = c;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; w++) {
    const int32_t v = wsum[w];
    base += w < wv ? v : 0;
    tot += v;
  }
  total = tot;
  return base + x - c;
}


// waves per SIMD a pass that evaluates the law is built for: 7 for the lean
// mixed-precision linear and Hertz laws (with the direct detection, over the
// 27-cell stencil; their registers just fit, without spills), the
// compiler's choice otherwise
template <int K, typename Real, int LAW>
constexpr int law_waves() {
  return K == 1 && sizeof(Real) == 4 && (LAW == DEM_LAW_LINEAR || LAW == DEM_LAW_HERTZ) ? 7 : 1;
}

// Steps 5-8 in one pass for the systems swept by the direct shape: each lane
// sweeps its particle's forward cells (the owned contacts go to the list),
// then each wave evaluates its particles' contacts one lane per contact
// (with_law; without it only the lists are built).
template <int K, typename Real, int LAW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(law_waves<K, Real, LAW>()))) void
k_contacts_direct(Layout L, StepCtl ctl, int32_t only_active, NbrBuf nb, const int32_t *__restrict__ scell,
                  const int32_t *__restrict__ cell_start, PairArgs a, int32_t with_law, int32_t *err) {
  __shared__ int32_t surv_all[kSurv * kBlock];
  __shared__ int32_t lst_all[kListStage * kBlock];
  __shared__ int32_t woff_all[kBlock / 64][65];
  int32_t k;
  const int32_t s = block_slot(L, k);
  const SysInfo &si = L.tab[k];
  if (si.tile != 0 || si.reach != K) return;  // another launch sweeps this system
  if (only_active && !is_active(ctl, k)) {    // a finished system keeps its lists and history
    if (with_law) carry_history<Real>(a, s);
    return;
  }
  int32_t cnt = 0;
  if (s >= 0) {
    const int32_t nx = si.g.nc[0], ny = si.g.nc[1], nz = si.g.nc[2];
    const int32_t cc = scell[s] - si.g.c0;
    const int32_t cx = cc % nx, cy = (cc / nx) % ny, cz = cc / (nx * ny);
    const DirectRows rows{nb.xq, cell_start, si.g.c0, nx, ny, nz, cy, cz};
    cnt = sweep_particle<kBlock, K>(rows, nb, sizeof(Real) == 8, L.n, s, si, cx, cy, cz, surv_all + threadIdx.x,
                                    lst_all + threadIdx.x, err);
  }
  if (!with_law) return;
  // where the block's contacts go: slot order, then k
  __shared__ int32_t wsum[kBlock / 64];
  int32_t tot;
  const int32_t off = block_exclusive_scan(cnt, wsum, tot);
  const int32_t q0 = (int32_t)cbase(blockIdx.x, a.nb.K) + off;
  set_hist_count<LAW>(a, s, cnt, q0);
  if (s >= 0) a.w.qs[s] = q0;
  const int32_t wave = (int32_t)(threadIdx.x >> 6);
  const HistAt own = owner_history<Real, LAW>(a, s);
  law_wave<Real, LAW>(a, si, L.bfirst[blockIdx.x] + wave * 64, cnt, lst_all + wave * 64, kBlock, woff_all[wave],
                      __shfl(q0, 0), own);
}

// The law pass of the systems swept by the wave and tiled shapes (their
// lists are in global memory), one lane per contact as in the direct pass.
template <typename Real, int LAW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(law_waves<1, Real, LAW>()))) void k_contact_law(
    PairArgs a, int32_t only_active) {
  __shared__ int32_t woff_all[kBlock / 64][65];
  int32_t k;
  const int32_t s = block_slot(a.L, k);
  const SysInfo &si = a.L.tab[k];
  if (si.tile == 0) return;  // evaluated by the direct pass
  if (only_active && !is_active(a.ctl, k)) {
    carry_history<Real>(a, s);
    return;
  }
  const int32_t cnt = s >= 0 ? a.nb.fcnt[s] : 0;
  __shared__ int32_t wsum[kBlock / 64];
  int32_t tot;
  const int32_t off = block_exclusive_scan(cnt, wsum, tot);
  const int32_t q0 = (int32_t)cbase(blockIdx.x, a.nb.K) + off;
  set_hist_count<LAW>(a, s, cnt, q0);
  if (s >= 0) a.w.qs[s] = q0;
  const int32_t wave = (int32_t)(threadIdx.x >> 6);
  const HistAt own = owner_history<Real, LAW>(a, s);
  law_wave<Real, LAW>(a, si, a.L.bfirst[blockIdx.x] + wave * 64, cnt, nullptr, 0, woff_all[wave], __shfl(q0, 0),
                      own);
}

// Step 1 drift x += dt v and Step 2 hash of the new position, written to
// the other position buffer
template <typename Real>
__device__ __forceinline__ void drift_hash_to(double x0, double y0, double z0, const PosBuf &out, int32_t i,
                                              const Real v[3], const Consts &c, const Grid &g, int32_t *cell,
                                              int32_t *err) {
#pragma clang fp contract(off)
  const double x = x0 + c.dt * (double)v[0];
  const double y = y0 + c.dt * (double)v[1];
  const double z = z0 + c.dt * (double)v[2];
  out.x[i] = x;
  out.y[i] = y;
  out.z[i] = z;
  int32_t cc;
  if (!hash_cell(g, x, y, z, &cc)) raise_err(err, ERR_DOMAIN);
  cell[i] = cc;
}

// --------------------------------------------------------------------------
// Step 7's sums, one lane per particle, in a fixed order (contacts with
// lower slots, ascending; with higher slots, ascending; walls), then in a
// time step the closing half kick and, when the system steps again in this
// call, the next step's opening kick, drift and hash.  The state goes to the
// other buffers.
//
// A particle's backward contacts (those with lower slots, owned and
// evaluated there) reach it through its kernel block: the law pass files
// each contact with the block its partner belongs to (one atomic per group
// of a wave's contacts with the same block), and the block sorts them to
// its particles in LDS.  Each particle then sums its own in ascending
// contact index, which is ascending owner slot: the order, and so the bits,
// do not depend on the order in which they were filed.  A block filed more
// than kBackCap of them finds them instead by scanning: each owner swept
// the forward half of its (2K + 1)^3 cells, so the owners of a particle's
// backward contacts lie in the mirror half, in slot order R = 1 + 2K + 2K^2
// runs of cells -- cells cx-K..cx of its own row (the slots below it),
// cells cx-K..cx+K of rows dy = -K..-1 of its plane and of rows dy = -K..K
// of planes dz = -K..-1 -- and each lane reads the list of every owner in
// the block's merged ranges of those runs.

constexpr int32_t kGatherStage = 512;  // backward records staged in LDS per block
constexpr int32_t kGatherRuns = 1 + 2 * kMaxReach + 2 * kMaxReach * kMaxReach;

// row offset of backward run h (h = 0: the own row)
__device__ __forceinline__ void back_row(int32_t h, int32_t K, int32_t &dy, int32_t &dz) {
  if (h <= K) {
    dy = -h;
    dz = 0;
  } else {
    const int32_t i = h - K - 1;
    dy = i % (2 * K + 1) - K;
    dz = -1 - i / (2 * K + 1);
  }
}

// the couple of the optional terms of contact q (XT: compiled in)
template <typename Real>
__device__ __forceinline__ void couple_of(const PairArgs &a, int64_t q, Real C[3]) {
  using V4 = typename Vec4T<Real>::type;
  const V4 cv = ((const V4 *)a.w.pc)[q];
  C[0] = cv.x;
  C[1] = cv.y;
  C[2] = cv.z;
}

template <typename Real, bool XT>
__global__ __launch_bounds__(kBlock) void k_gather(PairArgs a) {
  using V2 = typename Vec2T<Real>::type;
  constexpr int32_t kQueueBytes = kBackCap * 5;  // contact index and particle of each filed contact
  constexpr int32_t kRecBytes = 3 * kGatherStage * (int32_t)sizeof(V2);
  __shared__ int32_t bo[kBlock + 1];    // each particle's segment of bq
  __shared__ int32_t bq[kBackCap];      // the filed contacts' indices, by particle
  __shared__ int32_t lcnt[kBlock], lfill[kBlock];
  // first the filed contacts in arrival order, then the staged records
  __shared__ uint4 lds16[(kQueueBytes > kRecBytes ? kQueueBytes : kRecBytes) / 16 + 1];
  int32_t *hq = (int32_t *)lds16;
  uint8_t *hp = (uint8_t *)(hq + kBackCap);
  V2 *brec = (V2 *)lds16;
  __shared__ int32_t wlo[kGatherRuns], whi[kGatherRuns];  // each run's range (a crowded block)
  __shared__ int32_t rl[kGatherRuns], rh[kGatherRuns];    // merged
  __shared__ int32_t nmerged;
  __shared__ int32_t wsum[kBlock / 64];
  int32_t k;
  const int32_t s = block_slot(a.L, k);  // the block's particles are slots [s0, s0 + mblk), one system
  const SysInfo &si = a.L.tab[k];
  // the system's constants, grid and step control are read here, ahead of
  // every store, so that they are scalar loads (a store may alias them as
  // far as the compiler knows)
  const Consts c = si.c;
  const Grid g = si.g;
  const int32_t K = si.reach;
  const bool stepping = (a.mode & MODE_KICK) != 0;
  const int32_t step_now = stepping ? *a.ctl.step : 0, left_k = stepping ? a.ctl.left[k] : 0;
  const int32_t N = a.L.n;
  const int32_t s0 = a.L.bfirst[blockIdx.x], mblk = min(kBlock, si.p0 + si.n - s0);
  if (stepping && !(step_now < left_k)) {
    if (s < 0) return;
    const PState<Real> me = ((const PState<Real> *)a.nb.pst)[s];
    // a finished system: state unchanged; the next sort sees its current cells
#pragma unroll
    for (int q = 0; q < 3; q++) {
      ((Real *)a.vel_out.v[q])[s] = me.v[q];
      ((Real *)a.vel_out.w[q])[s] = me.w[q];
    }
    a.pos_out.x[s] = me.x;
    a.pos_out.y[s] = me.y;
    a.pos_out.z[s] = me.z;
    a.pos_out.r[s] = me.r;
    a.pos_out.id[s] = me.id & kIdMask;
    if (a.pos_out.mt) a.pos_out.mt[s] = me.id >> kMtShift;
    a.cell[s] = a.scell[s];
    return;
  }
  const int32_t nfiled = a.w.nback[blockIdx.x];
  const bool filed = nfiled <= kBackCap;
  // the particle's own contact count and first contact index are requested
  // ahead of the block's barriers, so that they have arrived when the sums
  // need them
  const int32_t nown = s >= 0 ? a.nb.fcnt[s] : 0;
  const int32_t q0 = s >= 0 ? a.w.qs[s] : 0;  // the particle's owned contacts
  lcnt[threadIdx.x] = 0;
  lfill[threadIdx.x] = 0;
  if (!filed) {
    // (a crowded block) per backward run, the slot range from the block's
    // first particle's run to its last one's.  A run outside the grid
    // stands for the empty range where it would lie (the start of the plane
    // for a row below it, the end of the plane for a row above it, the
    // system's first slot for a plane below it), so that the run ends grow
    // with the slot and the range covers the run of every particle in
    // between.
    const int32_t nx = g.nc[0], ny = g.nc[1];
    const int32_t R = 1 + 2 * K + 2 * K * K;
    if ((int32_t)threadIdx.x < R) {
      const int32_t h = (int32_t)threadIdx.x;
      int32_t dy, dz;
      back_row(h, K, dy, dz);
      const int32_t *cs = a.cell_start + g.c0;
      auto run_end = [&](int32_t t, bool start) {
        const int32_t cc = a.scell[t] - g.c0;
        const int32_t cx = cc % nx, yy = (cc / nx) % ny + dy, zz = cc / (nx * ny) + dz;
        if (zz < 0) return cs[0];
        if (yy < 0) return cs[zz * ny * nx];
        if (yy >= ny) return cs[(zz + 1) * ny * nx];
        if (start) return cs[(zz * ny + yy) * nx + max(cx - K, 0)];
        return h == 0 ? t : cs[(zz * ny + yy) * nx + min(cx + K, nx - 1) + 1];  // own row: owners below it
      };
      wlo[h] = run_end(s0, true);
      whi[h] = run_end(s0 + mblk - 1, false);
    }
    __syncthreads();
    // the ranges sorted and merged (one thread: at most 13)
    if (threadIdx.x == 0) {
      int32_t L[kGatherRuns], H[kGatherRuns], n = 0;
      for (int32_t h = 0; h < R; h++) {
        const int32_t lo = wlo[h], hi = whi[h];
        if (lo >= hi) continue;
        int32_t i = n++;
        for (; i > 0 && L[i - 1] > lo; i--) {
          L[i] = L[i - 1];
          H[i] = H[i - 1];
        }
        L[i] = lo;
        H[i] = hi;
      }
      int32_t nm = 0;
      for (int32_t i = 0; i < n; i++) {
        if (nm > 0 && L[i] <= rh[nm - 1]) {
          rh[nm - 1] = max(rh[nm - 1], H[i]);
        } else {
          rl[nm] = L[i];
          rh[nm] = H[i];
          nm++;
        }
      }
      nmerged = nm;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) a.w.nback[blockIdx.x] = 0;  // ready for the next evaluation's filing
  if (filed) {
    // the filed contacts, counted per particle
    const int2 *fb = a.w.back + (int64_t)blockIdx.x * kBackCap;
    // four entries per lane requested together (at most 4 kBlock are filed)
    static_assert(kBackCap <= 4 * kBlock, "four filed entries per lane at most");
    int2 f[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int32_t e = threadIdx.x + j * kBlock;
      if (e < nfiled) f[j] = fb[e];
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int32_t e = threadIdx.x + j * kBlock;
      if (e >= nfiled) break;
      const int32_t p = f[j].y - s0;
      if ((uint32_t)p < (uint32_t)mblk) {  // always (the block of the partner)
        atomicAdd(&lcnt[p], 1);
        hq[e] = f[j].x;
        hp[e] = (uint8_t)p;
      } else {
        hp[e] = 0;
        hq[e] = -1;
      }
    }
  }
  __syncthreads();
  const int32_t B = filed ? nfiled : INT32_MAX;
  const bool queued = filed, staged = B <= kGatherStage;
  const int32_t nbk = queued && s >= 0 ? lcnt[threadIdx.x] : 0;
  if (queued) {
    // the contacts by particle (in any order within a particle), then
    // their records into LDS with every lane on one
    int32_t tot;
    const int32_t off = block_exclusive_scan(nbk, wsum, tot);
    bo[threadIdx.x] = off;
    __syncthreads();
    for (int32_t e = threadIdx.x; e < B; e += kBlock) {
      const int32_t q = hq[e];
      if (q >= 0) {
        const int32_t p = hp[e];
        bq[bo[p] + atomicAdd(&lfill[p], 1)] = q;
      }
    }
    __syncthreads();
    if (staged) {
      for (int32_t e = threadIdx.x; e < tot; e += kBlock) {
        const V2 *p = (const V2 *)a.w.pf + 3 * (int64_t)bq[e];
        brec[3 * e] = p[0];
        brec[3 * e + 1] = p[1];
        brec[3 * e + 2] = p[2];
      }
    }
    __syncthreads();
  }
  if (s < 0) return;
  const PState<Real> me = ((const PState<Real> *)a.nb.pst)[s];
  const Real rs = (Real)me.r;
  Real F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  // contacts with lower partners, ascending by owner slot
  auto back = [&](int64_t q) {
    Real f[3], mm[3];
    get_record<Real>(a.w.pf, q, f, mm);
    F[0] -= f[0];
    F[1] -= f[1];
    F[2] -= f[2];
    T[0] += rs * mm[0];  // Eq. 3; the same n x F_t on both bodies
    T[1] += rs * mm[1];
    T[2] += rs * mm[2];
    if (XT) {  // the opposite of the owner's couple
      Real C[3];
      couple_of<Real>(a, q, C);
      T[0] -= C[0];
      T[1] -= C[1];
      T[2] -= C[2];
    }
  };
  if (queued) {
    // each next entry is the smallest above the previous one (an owner has
    // at most one contact with a given partner)
    const int32_t b0 = bo[threadIdx.x];
    int32_t prev = -1;
    for (int32_t i = 0; i < nbk; i++) {
      int32_t cur = INT32_MAX, at = b0;
      for (int32_t j = b0; j < b0 + nbk; j++) {
        const int32_t q = bq[j];
        if (q > prev && q < cur) {
          cur = q;
          at = j;
        }
      }
      prev = cur;
      if (staged) {
        const V2 r0 = brec[3 * at], r1 = brec[3 * at + 1], r2 = brec[3 * at + 2];
        F[0] -= r0.x;
        F[1] -= r0.y;
        F[2] -= r1.x;
        T[0] += rs * r1.y;  // Eq. 3; the same n x F_t on both bodies
        T[1] += rs * r2.x;
        T[2] += rs * r2.y;
        if (XT) {
          Real C[3];
          couple_of<Real>(a, cur, C);
          T[0] -= C[0];
          T[1] -= C[1];
          T[2] -= C[2];
        }
      } else {
        back(cur);
      }
    }
  } else {
    // a crowded block: the lane reads every owner's contacts itself, in
    // ascending slot order
    const int32_t nm = nmerged;
    for (int32_t i = 0; i < nm; i++)
      for (int32_t f = rl[i]; f < rh[i]; f++) {
        const int32_t q0 = a.w.qs[f], cn = a.nb.fcnt[f];
        for (int32_t j = 0; j < cn; j++)
          if (a.nb.nb[(int64_t)j * N + f] == s) back(q0 + j);
      }
  }
  double e_el = 0.0, dmax = 0.0;
  int32_t npair = 0, nwall = 0;
  const bool diag = (a.mode & MODE_DIAG) != 0;
  for (int32_t k0 = 0; k0 < nown; k0 += 2) {
    // the next two records requested together, then added in list order
    Real fb[2][3], mb[2][3];
#pragma unroll
    for (int j = 0; j < 2; j++)
      if (k0 + j < nown) get_record<Real>(a.w.pf, (int64_t)q0 + k0 + j, fb[j], mb[j]);
#pragma unroll
    for (int j = 0; j < 2; j++) {
      if (k0 + j >= nown) break;
      const int32_t k = k0 + j;
      const int64_t q = (int64_t)q0 + k;
      const Real *f = fb[j], *m = mb[j];
      F[0] += f[0];
      F[1] += f[1];
      F[2] += f[2];
      T[0] += rs * m[0];
      T[1] += rs * m[1];
      T[2] += rs * m[2];
      if (XT) {
        Real C[3];
        couple_of<Real>(a, q, C);
        T[0] += C[0];
        T[1] += C[1];
        T[2] += C[2];
      }
      if (diag) {
        e_el += a.w.pe[q];
        dmax = fmax(dmax, a.w.pd[q]);
        if (a.nb.nb[(int64_t)k * N + s] >= 0)
          npair++;
        else
          nwall++;
      }
    }
  }
  if (!(isfinite((double)F[0]) && isfinite((double)F[1]) && isfinite((double)F[2]) &&
        isfinite((double)T[0]) && isfinite((double)T[1]) && isfinite((double)T[2])))
    raise_err(a.err, ERR_NONFINITE);
  // the system steps again in this call: the forces stay in registers for
  // the fused kick; otherwise they are kept for the read-back and the next
  // call's opening kick
  const bool again = stepping && step_now + 1 < left_k;
  if (!again) {
#pragma unroll
    for (int q = 0; q < 3; q++) {
      ((Real *)a.F[q])[s] = F[q];
      ((Real *)a.T[q])[s] = T[q];
    }
  }
  if (stepping) {
    Real v[3] = {me.v[0], me.v[1], me.v[2]}, w[3] = {me.w[0], me.w[1], me.w[2]};
    const Real m = mass_of<Real>(c, rs);
    const Real I = (Real)0.4 * m * rs * rs;
    half_kick<Real>(c, m, I, F, T, v, w);
    if (again) {
      // the next step's Steps 1-2 with the same forces: the same operations
      // as k_kick_drift_hash, so fusing changes no bit
      half_kick<Real>(c, m, I, F, T, v, w);
      drift_hash_to(me.x, me.y, me.z, a.pos_out, s, v, c, g, a.cell, a.err);
    } else {
      a.pos_out.x[s] = me.x;  // its last step in this call: it stops here
      a.pos_out.y[s] = me.y;
      a.pos_out.z[s] = me.z;
      a.cell[s] = a.scell[s];
    }
    a.pos_out.r[s] = me.r;
    a.pos_out.id[s] = me.id & kIdMask;
    if (a.pos_out.mt) a.pos_out.mt[s] = me.id >> kMtShift;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      ((Real *)a.vel_out.v[q])[s] = v[q];
      ((Real *)a.vel_out.w[q])[s] = w[q];
    }
  }
  if (diag) {
    a.diag.e_el[s] = e_el;
    a.diag.npair[s] = npair;
    a.diag.nwall[s] = nwall;
    a.diag.dmax[s] = dmax;
  }
}

__global__ void k_step_end(StepCtl ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctl.step += 1;
}

// --------------------------------------------------------------------------
// Largest speed of each system (the at-rest test of Sec. 5's run: every
// particle's step dt |v| below a set value).  The maximum does not depend on
// the order of the updates, and a non-negative double orders like its bits.

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_max_speed(Layout L, VelBuf vb, unsigned long long *vmax) {
#pragma clang fp contract(off)
  int32_t k;
  const int32_t s = block_slot(L, k);
  double q = 0.0;
  if (s >= 0) {
    const double vx = (double)((const Real *)vb.v[0])[s], vy = (double)((const Real *)vb.v[1])[s],
                 vz = (double)((const Real *)vb.v[2])[s];
    q = sqrt(vx * vx + vy * vy + vz * vz);
  }
  // the block's largest, then one atomic per block
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) q = fmax(q, __shfl_xor(q, d));
  __shared__ double wmax[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int w = 1; w < kBlock / 64; w++) m = fmax(m, wmax[w]);
    atomicMax(vmax + k, (unsigned long long)__double_as_longlong(m));
  }
}

// --------------------------------------------------------------------------
// FP64 diagnostics: per-block partial sums in a fixed tree (a block holds
// one system's particles), then per system over its blocks in order

constexpr int kDiag = 10;

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_diag_partial(Layout L, PosBuf p, VelBuf vb, DiagBuf d) {
  __shared__ double sh[kDiag][kBlock];
  const int tid = threadIdx.x;
  int32_t k;
  const int32_t i = block_slot(L, k);
  const SysInfo &si = L.tab[k];
  double t[kDiag];
#pragma unroll
  for (int q = 0; q < kDiag; q++) t[q] = 0.0;
  if (i >= 0) {
    const Consts &c = si.c;
    const double r = (double)p.r[i];
    const double m = c.mass_c * r * r * r;
    const double I = 0.4 * m * r * r;
    double v[3], w[3];
    for (int q = 0; q < 3; q++) {
      v[q] = (double)((const Real *)vb.v[q])[i];
      w[q] = (double)((const Real *)vb.w[q])[i];
    }
    const double x[3] = {p.x[i], p.y[i], p.z[i]};
    for (int q = 0; q < 3; q++) t[q] = m * v[q];
    t[3] = 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    t[4] = 0.5 * I * (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double pe = 0.0;
    for (int q = 0; q < 3; q++) pe -= m * c.g[q] * (x[q] - si.g.lo[q]);
    t[5] = pe;
    t[6] = d.e_el[i];
    t[7] = (double)d.npair[i];
    t[8] = (double)d.nwall[i];
    t[9] = d.dmax[i];
  }
  for (int q = 0; q < kDiag; q++) sh[q][tid] = t[q];
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (tid < off) {
      for (int q = 0; q < 9; q++) sh[q][tid] += sh[q][tid + off];
      sh[9][tid] = fmax(sh[9][tid], sh[9][tid + off]);
    }
    __syncthreads();
  }
  if (tid == 0)
    for (int q = 0; q < kDiag; q++) d.partial[(int64_t)blockIdx.x * kDiag + q] = sh[q][0];
}

// one block per system; a system's blocks are consecutive, in system order
__global__ __launch_bounds__(kBlock) void k_diag_final(Layout L, DiagBuf d) {
  __shared__ double sh[kDiag][kBlock];
  const int tid = threadIdx.x;
  const int32_t k = blockIdx.x;
  const SysInfo &si = L.tab[k];
  int32_t b0 = 0;
  for (int32_t j = 0; j < k; j++) b0 += (L.tab[j].n + kBlock - 1) / kBlock;
  const int32_t nb = (si.n + kBlock - 1) / kBlock;
  double t[kDiag];
  for (int q = 0; q < kDiag; q++) t[q] = 0.0;
  for (int32_t b = tid; b < nb; b += kBlock) {
    for (int q = 0; q < 9; q++) t[q] += d.partial[(int64_t)(b0 + b) * kDiag + q];
    t[9] = fmax(t[9], d.partial[(int64_t)(b0 + b) * kDiag + 9]);
  }
  for (int q = 0; q < kDiag; q++) sh[q][tid] = t[q];
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (tid < off) {
      for (int q = 0; q < 9; q++) sh[q][tid] += sh[q][tid + off];
      sh[9][tid] = fmax(sh[9][tid], sh[9][tid + off]);
    }
    __syncthreads();
  }
  if (tid == 0)
    for (int q = 0; q < kDiag; q++) d.out[(int64_t)k * kDiag + q] = sh[q][0];
}

// --------------------------------------------------------------------------
// launchers

hipError_t launch_hash(const Layout &L, const PosBuf &p, int32_t *cell, int32_t *err, hipStream_t st) {
  if (L.n > 0) k_hash<<<L.nblocks, kBlock, 0, st>>>(L, p, cell, err);
  return hipGetLastError();
}

hipError_t launch_kick_drift_hash(int precision, const Layout &L, const StepCtl &ctl, const PosBuf &p,
                                  const VelBuf &v, void *const F[3], void *const T[3], const int32_t *scell,
                                  int32_t *cell, int32_t *err, hipStream_t st) {
  if (L.n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    k_kick_drift_hash<double><<<L.nblocks, kBlock, 0, st>>>(
        L, ctl, p, v, (const double *)F[0], (const double *)F[1], (const double *)F[2], (const double *)T[0],
        (const double *)T[1], (const double *)T[2], scell, cell, err);
  else
    k_kick_drift_hash<float><<<L.nblocks, kBlock, 0, st>>>(
        L, ctl, p, v, (const float *)F[0], (const float *)F[1], (const float *)F[2], (const float *)T[0],
        (const float *)T[1], (const float *)T[2], scell, cell, err);
  return hipGetLastError();
}

hipError_t launch_reorder(int precision, const Layout &L, const PosBuf &src, const VelBuf &vsrc, const PosBuf &dst,
                          const VelBuf &vdst, bool soa, const int32_t *perm, const int32_t *cell, int32_t *scell,
                          const NbrBuf &nb, const HistGen *old, hipStream_t st) {
  if (L.n <= 0) return hipSuccess;
  const int32_t *oc = old ? old->cnt : nullptr, *os = old ? old->start : nullptr;
  if (precision == DEM_PREC_FP64)
    k_reorder<double><<<L.nblocks, kBlock, 0, st>>>(L, src, vsrc, dst, vdst, soa ? 1 : 0, perm, cell, scell, nb,
                                                     oc, os);
  else
    k_reorder<float><<<L.nblocks, kBlock, 0, st>>>(L, src, vsrc, dst, vdst, soa ? 1 : 0, perm, cell, scell, nb,
                                                    oc, os);
  return hipGetLastError();
}

hipError_t launch_pack(int precision, const Layout &L, const PosBuf &p, const VelBuf &v, const NbrBuf &nb,
                       hipStream_t st) {
  if (L.n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    k_pack<double><<<L.nblocks, kBlock, 0, st>>>(L, p, v, nb);
  else
    k_pack<float><<<L.nblocks, kBlock, 0, st>>>(L, p, v, nb);
  return hipGetLastError();
}

hipError_t launch_xyzr(const Layout &L, const PosBuf &p, const NbrBuf &nb, hipStream_t st) {
  if (L.n > 0) k_xyzr<<<L.nblocks, kBlock, 0, st>>>(L, p, nb);
  return hipGetLastError();
}

template <typename Real, int LAW>
static hipError_t contacts_t(const Layout &L, const StepCtl *ctl, const NbrBuf &nb, const int32_t *scell,
                             const int32_t *cell_start, const PairArgs *a, int32_t *err, hipStream_t st,
                             hipEvent_t after_detect) {
  StepCtl none{nullptr, nullptr};
  const StepCtl c = ctl ? *ctl : none;
  const int32_t oa = ctl ? 1 : 0;
  PairArgs pa;
  if (a)
    pa = *a;
  else
    memset(&pa, 0, sizeof(pa));
  const int32_t wl = a ? 1 : 0;
  const bool f64 = sizeof(Real) == 8;
  if (L.ndirect > 0)
    k_contacts_direct<1, Real, LAW><<<L.nblocks, kBlock, 0, st>>>(L, c, oa, nb, scell, cell_start, pa, wl, err);
  if (L.ndirect2 > 0)
    k_contacts_direct<2, Real, LAW><<<L.nblocks, kBlock, 0, st>>>(L, c, oa, nb, scell, cell_start, pa, wl, err);
  if (L.nruns > 0)
    k_detect_cells<<<(L.nruns + kCellWaves - 1) / kCellWaves, kCellWaves * 64, 0, st>>>(L, c, oa, f64, nb, scell,
                                                                                        cell_start, err);
  if (L.ntiles > 0)
    k_detect_tiles<<<L.ntiles, kTileThreads, 0, st>>>(L, c, oa, f64, nb, scell, cell_start, err);
  if (after_detect) (void)hipEventRecord(after_detect, st);
  if (a && (L.nruns > 0 || L.ntiles > 0)) k_contact_law<Real, LAW><<<L.nblocks, kBlock, 0, st>>>(pa, oa);
  return hipGetLastError();
}

// the law's instantiation for one precision: the full form where a system
// may have a material-pair table or the pass computes diagnostics
template <int LAW>
static hipError_t contacts_law(bool f64, bool full, const Layout &L, const StepCtl *ctl, const NbrBuf &nb,
                               const int32_t *scell, const int32_t *cell_start, const PairArgs *a, int32_t *err,
                               hipStream_t st, hipEvent_t after_detect) {
  if (f64)
    return full ? contacts_t<double, LAW | kLawFull>(L, ctl, nb, scell, cell_start, a, err, st, after_detect)
                : contacts_t<double, LAW>(L, ctl, nb, scell, cell_start, a, err, st, after_detect);
  return full ? contacts_t<float, LAW | kLawFull>(L, ctl, nb, scell, cell_start, a, err, st, after_detect)
              : contacts_t<float, LAW>(L, ctl, nb, scell, cell_start, a, err, st, after_detect);
}

hipError_t launch_contacts(int precision, const Layout &L, const StepCtl *ctl, const NbrBuf &nb,
                           const int32_t *scell, const int32_t *cell_start, const PairArgs *a, int32_t *err,
                           hipStream_t st, hipEvent_t after_detect) {
  if (L.n <= 0) {
    if (after_detect) (void)hipEventRecord(after_detect, st);
    return hipSuccess;
  }
  const bool f64 = precision == DEM_PREC_FP64;
  // detection alone does not depend on the law
  const int law = a ? (a->law | (a->terms && a->law != DEM_LAW_SIMPLE ? kLawTerms : 0)) : DEM_LAW_LINEAR;
  const bool full = a && (a->mats != 0 || (a->mode & MODE_DIAG) != 0);
  switch (law) {
    case DEM_LAW_LINEAR | kLawTerms:
      return contacts_law<DEM_LAW_LINEAR | kLawTerms>(f64, full, L, ctl, nb, scell, cell_start, a, err, st,
                                                      after_detect);
    case DEM_LAW_HERTZ | kLawTerms:
      return contacts_law<DEM_LAW_HERTZ | kLawTerms>(f64, full, L, ctl, nb, scell, cell_start, a, err, st,
                                                     after_detect);
    case DEM_LAW_HERTZ:
      return contacts_law<DEM_LAW_HERTZ>(f64, full, L, ctl, nb, scell, cell_start, a, err, st, after_detect);
    case DEM_LAW_SIMPLE:
      return contacts_law<DEM_LAW_SIMPLE>(f64, full, L, ctl, nb, scell, cell_start, a, err, st, after_detect);
    default:
      return contacts_law<DEM_LAW_LINEAR>(f64, full, L, ctl, nb, scell, cell_start, a, err, st, after_detect);
  }
}

hipError_t launch_gather(int precision, const PairArgs &a, hipStream_t st) {
  if (a.L.n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64) {
    if (a.terms)
      k_gather<double, true><<<a.L.nblocks, kBlock, 0, st>>>(a);
    else
      k_gather<double, false><<<a.L.nblocks, kBlock, 0, st>>>(a);
  } else {
    if (a.terms)
      k_gather<float, true><<<a.L.nblocks, kBlock, 0, st>>>(a);
    else
      k_gather<float, false><<<a.L.nblocks, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_max_speed(int precision, const Layout &L, const VelBuf &v, unsigned long long *vmax,
                            hipStream_t st) {
  if (L.n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    k_max_speed<double><<<L.nblocks, kBlock, 0, st>>>(L, v, vmax);
  else
    k_max_speed<float><<<L.nblocks, kBlock, 0, st>>>(L, v, vmax);
  return hipGetLastError();
}

hipError_t launch_step_end(const StepCtl &ctl, hipStream_t st) {
  k_step_end<<<1, 64, 0, st>>>(ctl);
  return hipGetLastError();
}

hipError_t launch_diag_reduce(int precision, const Layout &L, const PosBuf &p, const VelBuf &v, const DiagBuf &d,
                              hipStream_t st) {
  if (L.n > 0) {
    if (precision == DEM_PREC_FP64)
      k_diag_partial<double><<<L.nblocks, kBlock, 0, st>>>(L, p, v, d);
    else
      k_diag_partial<float><<<L.nblocks, kBlock, 0, st>>>(L, p, v, d);
  }
  k_diag_final<<<L.S, kBlock, 0, st>>>(L, d);
  return hipGetLastError();
}

}  // namespace dem
