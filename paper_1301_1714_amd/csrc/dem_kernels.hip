// dem_kernels.hip -- HIP kernels of one DEM timestep for gfx950 (wave64).
//
// Steps of Sec. 4.2 and the kernels that run them:
//   Step 1       k_kick_drift_hash: opening half kick, drift and Step 2's
//                cell hash fused (one pass over the state)
//   Steps 2-3    k_count / scan / k_scatter / k_canon: counting sort by cell,
//                ties ordered by particle id, so SCM[j] = CM[SCCM[j]] (Eq. 11)
//                holds with one unique order; the paper's bitonic sort is
//                replaced by this O(N) sort (any correct sort of unique keys
//                gives the same permutation)
//   Step 4       k_reorder: gather every array into the sorted order, plus an
//                FP32 copy of (x - lo, r) for the detection prefilter
//   Steps 5-6    k_detect: one lane per sorted particle sweeps the forward
//                half of the 27 cells of Eq. 12 (each pair is tested once),
//                rejects with a conservative FP32 test and decides the rest
//                exactly in FP64; its contacts (ascending partner slot) and
//                walls form its list.  k_pairs / k_bwd: the lists become one
//                compact contact array (CSR by owner slot, from a scan) and a
//                backward index per partner (counting sort)
//   Steps 7-8    k_pair_force: one lane per contact -- every lane of a wave
//                evaluates a real contact, whatever the particles' contact
//                counts -- looks up the tangential history in the owner's
//                segment of the previous step's array and evaluates the law
//                (Eqs. 2-10, or Eq. 1) once per pair.  k_gather: one lane per
//                particle sums its contacts in a fixed order (lower partners,
//                higher partners, walls; no atomics) and applies the closing
//                half kick
// No step is a dense contraction, so nothing here uses the matrix cores.
#include <math.h>

#include "dem_internal.h"

namespace dem {

constexpr int kBlock = 256;

__device__ __forceinline__ void raise_err(int32_t *err, int32_t bit) { atomicOr(err, bit); }

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

// Step 2: cell of a position (Sec. 4.1).  Returns false when the particle is
// more than one cell outside the box (or not finite).
__device__ __forceinline__ bool hash_cell(const Grid &g, double x, double y, double z, int32_t *cell) {
#pragma clang fp contract(off)
  const double p[3] = {x, y, z};
  int32_t ijk[3];
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    double u = (p[a] - g.lo[a]) * g.sc[a];
    ok = ok && (u >= -1.0 && u < (double)g.nc[a] + 1.0);
    double f = floor(u);
    int32_t i = f < 0.0 ? 0 : (f > (double)(g.nc[a] - 1) ? g.nc[a] - 1 : (int32_t)f);
    ijk[a] = i;
  }
  *cell = ijk[0] + g.nc[0] * (ijk[1] + g.nc[1] * ijk[2]);
  return ok;
}

template <typename Real>
__device__ __forceinline__ Real mass_of(const Consts &c, Real r) {
  return (Real)c.mass_c * r * r * r;
}

// --------------------------------------------------------------------------
// Steps 1-2

__global__ __launch_bounds__(kBlock) void k_hash(PosBuf p, int32_t n, Grid g, int32_t *cell, int32_t *err) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int32_t c;
  if (!hash_cell(g, p.x[i], p.y[i], p.z[i], &c)) raise_err(err, ERR_DOMAIN);
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
__global__ __launch_bounds__(kBlock) void k_kick_drift_hash(PosBuf p, VelBuf vb, const Real *__restrict__ Fx,
                                                            const Real *__restrict__ Fy,
                                                            const Real *__restrict__ Fz,
                                                            const Real *__restrict__ Tx,
                                                            const Real *__restrict__ Ty,
                                                            const Real *__restrict__ Tz, int32_t n, Consts c,
                                                            Grid g, int32_t *cell, int32_t *err) {
#pragma clang fp contract(off)
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  Real *V[3] = {(Real *)vb.v[0], (Real *)vb.v[1], (Real *)vb.v[2]};
  Real *Wv[3] = {(Real *)vb.w[0], (Real *)vb.w[1], (Real *)vb.w[2]};
  const Real r = (Real)p.r[i];
  const Real m = mass_of<Real>(c, r);
  const Real I = (Real)0.4 * m * r * r;
  Real v[3] = {V[0][i], V[1][i], V[2][i]};
  Real w[3] = {Wv[0][i], Wv[1][i], Wv[2][i]};
  const Real F[3] = {Fx[i], Fy[i], Fz[i]};
  const Real T[3] = {Tx[i], Ty[i], Tz[i]};
  half_kick<Real>(c, m, I, F, T, v, w);
#pragma unroll
  for (int k = 0; k < 3; k++) {
    V[k][i] = v[k];
    Wv[k][i] = w[k];
  }
  drift_hash(p, i, v, c, g, cell, err);
}

// --------------------------------------------------------------------------
// Step 3: counting sort by cell, then a canonical order (by id) inside cells

__global__ __launch_bounds__(kBlock) void k_fill(int32_t *a, int64_t len, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < len) a[i] = value;
}

// Cell counts and each particle's rank in its cell.  The input is in the
// previous step's sorted order, so neighbouring lanes mostly share a cell:
// each run of equal cells within a wave takes one atomic for its length.
__global__ __launch_bounds__(kBlock) void k_count(const int32_t *__restrict__ cell, int32_t *__restrict__ rank,
                                                  int32_t *counts, int32_t n) {
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

// insertion sort of each cell's slots by particle id (cells hold a handful)
__global__ __launch_bounds__(kBlock) void k_canon(const int32_t *__restrict__ cell_start,
                                                  const int32_t *__restrict__ id_old, int32_t *perm,
                                                  int64_t ncell) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell) return;
  const int32_t beg = cell_start[c], end = cell_start[c + 1];
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

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_sort(const int32_t *cell, const int32_t *id_old, int32_t n, int64_t ncell, int32_t *counts,
                       int32_t *rank, int32_t *cell_start, int32_t *perm, const ScanScratch &sc,
                       hipStream_t st) {
  k_fill<<<blocks_for(ncell), kBlock, 0, st>>>(counts, ncell, 0);
  if (n > 0) k_count<<<blocks_for(n), kBlock, 0, st>>>(cell, rank, counts, n);
  hipError_t e = scan_exclusive(counts, cell_start, ncell, sc, 0, st);
  if (e != hipSuccess) return e;
  k_scan_total<<<1, 64, 0, st>>>(counts, cell_start, ncell);
  if (n > 0) {
    k_scatter<<<blocks_for(n), kBlock, 0, st>>>(cell, rank, cell_start, perm, n);
    k_canon<<<blocks_for(ncell), kBlock, 0, st>>>(cell_start, id_old, perm, ncell);
  }
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Step 4: gather into the sorted order

__device__ __forceinline__ float4 make_xyzr(const Grid &g, double x, double y, double z, float r) {
  return make_float4((float)(x - g.lo[0]), (float)(y - g.lo[1]), (float)(z - g.lo[2]), r);
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_reorder(PosBuf src, VelBuf vsrc, PosBuf dst, VelBuf vdst,
                                                    const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ cell, int32_t *__restrict__ scell,
                                                    float4 *__restrict__ xyzr, Grid g, int32_t n) {
  const int32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n) return;
  const int32_t p = perm[s];
  const double x = src.x[p], y = src.y[p], z = src.z[p];
  const float r = src.r[p];
  dst.x[s] = x;
  dst.y[s] = y;
  dst.z[s] = z;
  dst.r[s] = r;
  dst.id[s] = src.id[p];
  xyzr[s] = make_xyzr(g, x, y, z, r);
#pragma unroll
  for (int k = 0; k < 3; k++) {
    ((Real *)vdst.v[k])[s] = ((const Real *)vsrc.v[k])[p];
    ((Real *)vdst.w[k])[s] = ((const Real *)vsrc.w[k])[p];
  }
  scell[s] = cell[p];
}


__global__ __launch_bounds__(kBlock) void k_xyzr(PosBuf p, float4 *__restrict__ xyzr, Grid g, int32_t n) {
  const int32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n) return;
  xyzr[s] = make_xyzr(g, p.x[s], p.y[s], p.z[s], p.r[s]);
}

// --------------------------------------------------------------------------
// Steps 5-6: contact detection over the forward half of the 27-cell stencil.
// A pair in neighbouring cells is tested by the particle whose cell comes
// first in (z, y, x) order; a pair in one cell by the lower slot.  Every
// partner found this way has a higher slot, so the list comes out ascending
// without atomics.

constexpr int kSurv = 16;  // LDS survivor slots per lane

// exact FP64 decision on one prefilter survivor (Steps 6-7: the contact test)
__device__ __forceinline__ void exact_and_record(const NbrBuf &nb, const PosBuf &pos, int32_t N, int32_t s,
                                                 float ri, double xi, double yi, double zi, int32_t t,
                                                 int32_t &nf) {
  const double ex = pos.x[t] - xi, ey = pos.y[t] - yi, ez = pos.z[t] - zi;
  const double S = (double)ri + (double)pos.r[t];
  if (!(dist2_exact(ex, ey, ez) < sq_exact(S))) return;
  if (nf < kListCap) nb.nb[(int64_t)nf * N + s] = t;
  nf++;
}

// Prefilter one slot range; survivors wait in the lane's LDS slots so that
// the rare exact test does not sit inside the candidate loop (where any one
// lane taking it would hold the whole wave).  A lane whose slots fill up
// drains them itself, in order.
__device__ __forceinline__ void prefilter_range(const NbrBuf &nb, const PosBuf &pos, int32_t N, int32_t s,
                                                const float4 p, double xi, double yi, double zi, int32_t beg,
                                                int32_t end, int32_t *surv, int32_t &ns, int32_t &nf) {
  for (int32_t t = beg; t < end; t++) {
    const float4 q = nb.xyzr[t];
    const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
    const float sf = p.w + q.w + nb.eps;
    if (dx * dx + dy * dy + dz * dz < sf * sf) {
      if (ns == kSurv) {
        for (int k = 0; k < kSurv; k++) exact_and_record(nb, pos, N, s, p.w, xi, yi, zi, surv[k * kBlock], nf);
        ns = 0;
      }
      surv[ns * kBlock] = t;
      ns++;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_detect(PosBuf pos, NbrBuf nb, const int32_t *__restrict__ scell,
                                                   const int32_t *__restrict__ cell_start, Grid g,
                                                   uint32_t wall_mask, int32_t n, int32_t *err) {
  __shared__ int32_t surv_all[kSurv * kBlock];
  const int32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n) return;
  int32_t *surv = surv_all + threadIdx.x;  // slot k at surv[k * kBlock]
  const float4 p = nb.xyzr[s];
  const double xi = pos.x[s], yi = pos.y[s], zi = pos.z[s];
  const int32_t nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
  const int32_t cc = scell[s];
  const int32_t cx = cc % nx, cy = (cc / nx) % ny, cz = cc / (nx * ny);
  const int32_t x0 = cx > 0 ? cx - 1 : 0, x1 = cx < nx - 1 ? cx + 1 : nx - 1;
  int32_t nf = 0, ns = 0;
  // own row: the rest of the own cell and the next cell along x
  const int32_t row0 = (cz * ny + cy) * nx;
  prefilter_range(nb, pos, n, s, p, xi, yi, zi, s + 1, cell_start[row0 + x1 + 1], surv, ns, nf);
  // next row along y in the same plane
  if (cy + 1 < ny) {
    const int32_t row = (cz * ny + cy + 1) * nx;
    prefilter_range(nb, pos, n, s, p, xi, yi, zi, cell_start[row + x0], cell_start[row + x1 + 1], surv, ns, nf);
  }
  // the three rows of the next plane along z
  if (cz + 1 < nz) {
    for (int32_t dy = -1; dy <= 1; dy++) {
      const int32_t yy = cy + dy;
      if (yy < 0 || yy >= ny) continue;
      const int32_t row = ((cz + 1) * ny + yy) * nx;
      prefilter_range(nb, pos, n, s, p, xi, yi, zi, cell_start[row + x0], cell_start[row + x1 + 1], surv, ns,
                      nf);
    }
  }
  // exact tests of the survivors, in slot order
  for (int32_t k = 0; k < ns; k++) exact_and_record(nb, pos, n, s, p.w, xi, yi, zi, surv[k * kBlock], nf);
  // Step 8: walls, particles of infinite radius, after the pairs
  if (wall_mask) {
    const double xs[3] = {xi, yi, zi};
    const double rid = (double)p.w;
    for (int w = 0; w < 6; w++) {
      if (!((wall_mask >> w) & 1)) continue;
      const int ax = w >> 1;
      const double gap = (w & 1) ? (g.hi[ax] - xs[ax]) : (xs[ax] - g.lo[ax]);
      if (gap < rid) {
        if (nf < kListCap) nb.nb[(int64_t)nf * n + s] = -1 - w;
        nf++;
      }
    }
  }
  if (nf > kListCap) raise_err(err, ERR_OVERFLOW);
  nb.cnt[s] = nf < kListCap ? nf : kListCap;
}

// The lists become the compact contact array of `gen` (offsets from a scan of
// the counts); each pair also counts towards its partner's backward list.
__global__ __launch_bounds__(kBlock) void k_pairs(NbrBuf nb, PosBuf pos, PairGen gen, PairWork w, int32_t n,
                                                  int32_t *err) {
  const int32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n) return;
  const int32_t cnt = nb.cnt[s];
  const int64_t base = gen.ofs[s];
  if (base + cnt > w.Pcap) raise_err(err, ERR_OVERFLOW);  // contacts past the capacity are dropped
  for (int32_t k = 0; k < cnt; k++) {
    const int32_t t = nb.nb[(int64_t)k * n + s];
    const int64_t q = base + k;
    if (q >= w.Pcap) break;
    gen.s[q] = s;
    gen.t[q] = t;
    gen.key[q] = t >= 0 ? pos.id[t] : t;
    if (t >= 0) w.brank[q] = atomicAdd(&w.bcnt[t], 1);
  }
}

__device__ __forceinline__ int32_t num_pairs(const PairGen &gen, int32_t n, int64_t cap) {
  const int32_t P = gen.ofs[n];
  return (int64_t)P < cap ? P : (int32_t)cap;
}

// backward index: contact q is filed under its partner at the rank its
// count drew (arrival order; the gather sorts each short segment)
__global__ __launch_bounds__(kBlock) void k_bwd(PairGen gen, PairWork w, int32_t n) {
  const int32_t P = num_pairs(gen, n, w.Pcap);
  for (int32_t q = blockIdx.x * kBlock + threadIdx.x; q < P; q += gridDim.x * kBlock) {
    const int32_t t = gen.t[q];
    if (t < 0) continue;
    w.bwd[w.bofs[t] + w.brank[q]] = q;
  }
}

// fixed-size bitonic network on registers (indices are compile-time)
template <int M>
__device__ __forceinline__ void bitonic_sort(int32_t (&L)[M]) {
#pragma unroll
  for (int k = 2; k <= M; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < M; i++) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const int32_t u = L[i], v = L[l];
          const bool sw = up ? (u > v) : (u < v);
          L[i] = sw ? v : u;
          L[l] = sw ? u : v;
        }
      }
    }
  }
}

template <int M>
__device__ __forceinline__ void sort_small(int32_t *list, int32_t cnt) {
  int32_t L[M];
#pragma unroll
  for (int i = 0; i < M; i++) L[i] = i < cnt ? list[i] : INT32_MAX;
  bitonic_sort<M>(L);
#pragma unroll
  for (int i = 0; i < M; i++)
    if (i < cnt) list[i] = L[i];
}

// ascending order of a short contiguous list (entries arrived by atomics)
__device__ __forceinline__ void sort_list(int32_t *list, int32_t cnt) {
  if (cnt <= 1) return;
  if (cnt <= 4) {
    sort_small<4>(list, cnt);
  } else if (cnt <= 8) {
    sort_small<8>(list, cnt);
  } else if (cnt <= 16) {
    sort_small<16>(list, cnt);
  } else {
    for (int32_t k = 1; k < cnt; k++) {
      const int32_t v = list[k];
      int32_t j = k - 1;
      while (j >= 0 && list[j] > v) {
        list[j + 1] = list[j];
        j--;
      }
      list[j + 1] = v;
    }
  }
}

// --------------------------------------------------------------------------
// Steps 7-8: contact law

template <typename Real>
struct LawOut {
  Real F[3];     // force on the first body
  Real Ft[3];    // its tangential part (sets the torque of Eq. 3)
  Real dtn[3];   // new tangential displacement (Eq. 7, after Eq. 5)
  Real kn, kt;   // stiffness used (elastic-energy diagnostic)
};

// One contact seen from body a: n (unit, a -> partner), overlap delta,
// effective radius R and mass M, relative velocity v = v_a - v_b, spin term
// r_a w_a + r_b w_b, previous tangential displacement h.
template <typename Real, int LAW>
__device__ __forceinline__ void contact_law(const Consts &c, const Real n[3], Real delta, Real R, Real M,
                                            const Real v[3], const Real spin[3], const Real h[3],
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
#pragma unroll
    for (int k = 0; k < 3; k++) {
      o.F[k] = -(Real)c.k_sp * delta * n[k] - (Real)c.k_da * v[k] - (Real)c.k_sh * vt[k];
      o.Ft[k] = 0;
      o.dtn[k] = 0;
    }
    o.kn = (Real)c.k_sp;
    o.kt = 0;
    return;
  }
  Real kn, kt;
  if (LAW == DEM_LAW_HERTZ) {  // Eqs. 8-9
    const Real q = sqrt(delta * R);
    kn = (Real)c.kn * q;
    kt = (Real)c.kt * q;
  } else {
    kn = (Real)c.kn;
    kt = (Real)c.kt;
  }
  const Real eta = (Real)c.alpha * sqrt(kn * M);  // Eq. 10
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
  const Real lim = (Real)c.mu * fnn;
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
}

template <typename Real, int LAW>
__device__ __forceinline__ double elastic_energy(const Consts &c, Real delta, Real R, const LawOut<Real> &o,
                                                 const Real h[3]) {
  const double d = (double)delta;
  const double hh = (double)h[0] * h[0] + (double)h[1] * h[1] + (double)h[2] * h[2];
  if (LAW == DEM_LAW_SIMPLE) return 0.5 * c.k_sp * d * d;
  if (LAW == DEM_LAW_HERTZ) return 0.4 * c.kn * sqrt((double)R) * pow(d, 2.5) + 0.5 * (double)o.kt * hh;
  return 0.5 * (double)o.kn * d * d + 0.5 * (double)o.kt * hh;
}

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

// committed tangential displacement of the contact with history key `key`
// in segment `owner` of the previous array (zero for a new contact)
template <typename Real>
__device__ __forceinline__ void hist_lookup(const PairGen &old, int64_t cap, int32_t owner, int32_t key,
                                            Real h[3]) {
  using V4 = typename Vec4T<Real>::type;
  h[0] = h[1] = h[2] = 0;
  int64_t q = old.ofs[owner];
  const int64_t e = old.ofs[owner + 1] < cap ? old.ofs[owner + 1] : cap;
  for (; q < e; q++) {
    if (old.key[q] == key) {
      const V4 d = ((const V4 *)old.dt)[q];
      h[0] = d.x;
      h[1] = d.y;
      h[2] = d.z;
      break;
    }
  }
}

// One lane per contact: the law of Eqs. 2-10 (or Eq. 1) evaluated once per
// pair in the canonical orientation (lower particle id first), stored as the
// force on the owner and n x F_t.
template <typename Real, int LAW>
__global__ __launch_bounds__(kBlock) void k_pair_force(PairArgs a) {
  using V4 = typename Vec4T<Real>::type;
  const Consts &c = a.c;
  const int32_t P = num_pairs(a.cur, a.n, a.w.Pcap);
  const Real *VI[3] = {(const Real *)a.vel_in.v[0], (const Real *)a.vel_in.v[1], (const Real *)a.vel_in.v[2]};
  const Real *WI[3] = {(const Real *)a.vel_in.w[0], (const Real *)a.vel_in.w[1], (const Real *)a.vel_in.w[2]};
  const bool old_perm = (a.mode & MODE_OLD_PERM) != 0;
  const bool write_hist = (a.mode & MODE_WRITE_HIST) != 0 && LAW != DEM_LAW_SIMPLE;
  const bool diag = (a.mode & MODE_DIAG) != 0;
  for (int32_t q = blockIdx.x * kBlock + threadIdx.x; q < P; q += gridDim.x * kBlock) {
    const int32_t s = a.cur.s[q], t = a.cur.t[q];
    const double xs = a.pos.x[s], ys = a.pos.y[s], zs = a.pos.z[s];
    const float rsf = a.pos.r[s];
    const Real rs = (Real)rsf;
    const Real ms = mass_of<Real>(c, rs);
    const Real vs[3] = {VI[0][s], VI[1][s], VI[2][s]};
    const Real ws[3] = {WI[0][s], WI[1][s], WI[2][s]};
    const int32_t ps = old_perm ? a.perm[s] : s;
    LawOut<Real> o;
    Real n[3], h[3] = {0, 0, 0}, Fown[3], delta, R;
    if (t >= 0) {
      const int32_t ids = a.pos.id[s], idt = a.pos.id[t];
      const double dx = a.pos.x[t] - xs, dy = a.pos.y[t] - ys, dz = a.pos.z[t] - zs;
      const double d2 = dist2_exact(dx, dy, dz);
      const double S = (double)rsf + (double)a.pos.r[t];
      const Real rt = (Real)a.pos.r[t];
      const Real vt_[3] = {VI[0][t], VI[1][t], VI[2][t]};
      const Real wt_[3] = {WI[0][t], WI[1][t], WI[2][t]};
      const Real mt = mass_of<Real>(c, rt);
      const bool low = ids < idt;  // s is the canonical first body
      const Real ra = low ? rs : rt, rb = low ? rt : rs;
      const Real ma = low ? ms : mt, mb = low ? mt : ms;
      const double ex = low ? dx : -dx, ey = low ? dy : -dy, ez = low ? dz : -dz;
      const Real dd = sqrt((Real)d2);
      const Real invd = (Real)1 / dd;
      n[0] = (Real)ex * invd;
      n[1] = (Real)ey * invd;
      n[2] = (Real)ez * invd;
      delta = (Real)(sq_exact(S) - d2) / ((Real)S + dd);
      R = ra * rb / (ra + rb);
      const Real M = ma * mb / (ma + mb);
      Real v[3], spin[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const Real va = low ? vs[k] : vt_[k], vb = low ? vt_[k] : vs[k];
        const Real wa = low ? ws[k] : wt_[k], wb = low ? wt_[k] : ws[k];
        v[k] = va - vb;
        spin[k] = ra * wa + rb * wb;
      }
      if (LAW != DEM_LAW_SIMPLE) {
        // the previous step filed this pair under its lower slot then
        const int32_t pt = old_perm ? a.perm[t] : t;
        hist_lookup<Real>(a.old, a.w.Pcap, ps < pt ? ps : pt, ps < pt ? idt : ids, h);
      }
      contact_law<Real, LAW>(c, n, delta, R, M, v, spin, h, o);
#pragma unroll
      for (int k = 0; k < 3; k++) Fown[k] = low ? o.F[k] : -o.F[k];
    } else {
      // Step 8: wall -1 - t, a particle of infinite radius
      const int w = -1 - t;
      const int ax = w >> 1;
      const double xw[3] = {xs, ys, zs};
      const double gap = (w & 1) ? (a.grid.hi[ax] - xw[ax]) : (xw[ax] - a.grid.lo[ax]);
      n[0] = n[1] = n[2] = 0;
      n[ax] = (w & 1) ? (Real)1 : (Real)-1;
      delta = (Real)((double)rsf - gap);
      R = rs;
      Real spin[3];
#pragma unroll
      for (int k = 0; k < 3; k++) spin[k] = rs * ws[k];
      if (LAW != DEM_LAW_SIMPLE) hist_lookup<Real>(a.old, a.w.Pcap, ps, t, h);
      contact_law<Real, LAW>(c, n, delta, rs, ms, vs, spin, h, o);
#pragma unroll
      for (int k = 0; k < 3; k++) Fown[k] = o.F[k];
    }
    V4 f, tq;
    f.x = Fown[0];
    f.y = Fown[1];
    f.z = Fown[2];
    f.w = 0;
    tq.x = n[1] * o.Ft[2] - n[2] * o.Ft[1];
    tq.y = n[2] * o.Ft[0] - n[0] * o.Ft[2];
    tq.z = n[0] * o.Ft[1] - n[1] * o.Ft[0];
    tq.w = 0;
    ((V4 *)a.w.pf)[2 * (int64_t)q] = f;
    ((V4 *)a.w.pf)[2 * (int64_t)q + 1] = tq;
    if (write_hist) {
      V4 d;
      d.x = o.dtn[0];
      d.y = o.dtn[1];
      d.z = o.dtn[2];
      d.w = 0;
      ((V4 *)a.cur.dt)[q] = d;
    }
    if (diag) {
      a.w.pe[q] = elastic_energy<Real, LAW>(c, delta, R, o, h);
      a.w.pd[q] = (double)delta;
    }
  }
}

// One lane per particle: contact sums in a fixed order (contacts with lower
// slots, ascending; with higher slots, ascending; walls), then the closing
// half kick of Step 1.
template <typename Real>
__global__ __launch_bounds__(kBlock) void k_gather(PairArgs a) {
  using V4 = typename Vec4T<Real>::type;
  const int32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= a.n) return;
  const Consts &c = a.c;
  const int64_t cap = a.w.Pcap;
  const Real rs = (Real)a.pos.r[s];
  const V4 *pf = (const V4 *)a.w.pf;  // contact q: force at 2q, n x F_t at 2q + 1
  Real F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  const int32_t b0 = a.w.bofs[s], b1 = a.w.bofs[s + 1];
  const int32_t nb = (int64_t)b1 <= cap ? b1 - b0 : 0;
  sort_list(a.w.bwd + b0, nb);
  for (int32_t k = 0; k < nb; k++) {
    const int32_t q = a.w.bwd[b0 + k];
    const V4 f = pf[2 * (int64_t)q], m = pf[2 * (int64_t)q + 1];
    F[0] -= f.x;
    F[1] -= f.y;
    F[2] -= f.z;
    T[0] += rs * m.x;  // Eq. 3; the same n x F_t on both bodies
    T[1] += rs * m.y;
    T[2] += rs * m.z;
  }
  const int64_t f0 = a.cur.ofs[s];
  const int64_t f1 = a.cur.ofs[s + 1] < cap ? a.cur.ofs[s + 1] : cap;
  double e_el = 0.0, dmax = 0.0;
  int32_t npair = 0, nwall = 0;
  const bool diag = (a.mode & MODE_DIAG) != 0;
  for (int64_t q = f0; q < f1; q++) {
    const V4 f = pf[2 * q], m = pf[2 * q + 1];
    F[0] += f.x;
    F[1] += f.y;
    F[2] += f.z;
    T[0] += rs * m.x;
    T[1] += rs * m.y;
    T[2] += rs * m.z;
    if (diag) {
      e_el += a.w.pe[q];
      dmax = fmax(dmax, a.w.pd[q]);
      if (a.cur.t[q] >= 0)
        npair++;
      else
        nwall++;
    }
  }
  if (!(isfinite((double)F[0]) && isfinite((double)F[1]) && isfinite((double)F[2]) &&
        isfinite((double)T[0]) && isfinite((double)T[1]) && isfinite((double)T[2])))
    raise_err(a.err, ERR_NONFINITE);
#pragma unroll
  for (int k = 0; k < 3; k++) {
    ((Real *)a.F[k])[s] = F[k];
    ((Real *)a.T[k])[s] = T[k];
  }
  if (a.mode & MODE_KICK) {
    const Real *VI[3] = {(const Real *)a.vel_in.v[0], (const Real *)a.vel_in.v[1], (const Real *)a.vel_in.v[2]};
    const Real *WI[3] = {(const Real *)a.vel_in.w[0], (const Real *)a.vel_in.w[1], (const Real *)a.vel_in.w[2]};
    Real v[3] = {VI[0][s], VI[1][s], VI[2][s]}, w[3] = {WI[0][s], WI[1][s], WI[2][s]};
    const Real m = mass_of<Real>(c, rs);
    const Real I = (Real)0.4 * m * rs * rs;
    half_kick<Real>(c, m, I, F, T, v, w);
    if (a.mode & MODE_DRIFT) {
      // the next step's Steps 1-2 with the same forces: the same operations
      // as k_kick_drift_hash, so fusing changes no bit
      half_kick<Real>(c, m, I, F, T, v, w);
      drift_hash(a.pos, s, v, c, a.grid, a.cell, a.err);
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
      ((Real *)a.vel_out.v[k])[s] = v[k];
      ((Real *)a.vel_out.w[k])[s] = w[k];
    }
  }
  if (diag) {
    a.diag.e_el[s] = e_el;
    a.diag.npair[s] = npair;
    a.diag.nwall[s] = nwall;
    a.diag.dmax[s] = dmax;
  }
}

// --------------------------------------------------------------------------
// FP64 diagnostics: per-block partial sums in a fixed tree, then one block

constexpr int kDiag = 10;

int diag_blocks(int32_t n) {
  int b = (int)((n + kBlock - 1) / kBlock);
  return b < 1 ? 1 : b;
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_diag_partial(PosBuf p, VelBuf vb, DiagBuf d, int32_t n, Consts c,
                                                         Grid g) {
  __shared__ double sh[kDiag][kBlock];
  const int tid = threadIdx.x;
  const int32_t i = blockIdx.x * kBlock + tid;
  double t[kDiag];
#pragma unroll
  for (int k = 0; k < kDiag; k++) t[k] = 0.0;
  if (i < n) {
    const double r = (double)p.r[i];
    const double m = c.mass_c * r * r * r;
    const double I = 0.4 * m * r * r;
    double v[3], w[3];
    for (int k = 0; k < 3; k++) {
      v[k] = (double)((const Real *)vb.v[k])[i];
      w[k] = (double)((const Real *)vb.w[k])[i];
    }
    const double x[3] = {p.x[i], p.y[i], p.z[i]};
    for (int k = 0; k < 3; k++) t[k] = m * v[k];
    t[3] = 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    t[4] = 0.5 * I * (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double pe = 0.0;
    for (int k = 0; k < 3; k++) pe -= m * c.g[k] * (x[k] - g.lo[k]);
    t[5] = pe;
    t[6] = d.e_el[i];
    t[7] = (double)d.npair[i];
    t[8] = (double)d.nwall[i];
    t[9] = d.dmax[i];
  }
  for (int k = 0; k < kDiag; k++) sh[k][tid] = t[k];
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (tid < off) {
      for (int k = 0; k < 9; k++) sh[k][tid] += sh[k][tid + off];
      sh[9][tid] = fmax(sh[9][tid], sh[9][tid + off]);
    }
    __syncthreads();
  }
  if (tid == 0)
    for (int k = 0; k < kDiag; k++) d.partial[(int64_t)blockIdx.x * kDiag + k] = sh[k][0];
}

__global__ __launch_bounds__(kBlock) void k_diag_final(DiagBuf d, int nblocks) {
  __shared__ double sh[kDiag][kBlock];
  const int tid = threadIdx.x;
  double t[kDiag];
  for (int k = 0; k < kDiag; k++) t[k] = 0.0;
  for (int b = tid; b < nblocks; b += kBlock) {
    for (int k = 0; k < 9; k++) t[k] += d.partial[(int64_t)b * kDiag + k];
    t[9] = fmax(t[9], d.partial[(int64_t)b * kDiag + 9]);
  }
  for (int k = 0; k < kDiag; k++) sh[k][tid] = t[k];
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (tid < off) {
      for (int k = 0; k < 9; k++) sh[k][tid] += sh[k][tid + off];
      sh[9][tid] = fmax(sh[9][tid], sh[9][tid + off]);
    }
    __syncthreads();
  }
  if (tid == 0)
    for (int k = 0; k < kDiag; k++) d.out[k] = sh[k][0];
}

// --------------------------------------------------------------------------
// launchers

hipError_t launch_hash(const PosBuf &p, int32_t n, const Grid &g, int32_t *cell, int32_t *err, hipStream_t st) {
  if (n > 0) k_hash<<<blocks_for(n), kBlock, 0, st>>>(p, n, g, cell, err);
  return hipGetLastError();
}

template <typename Real>
static void kdh_t(const PosBuf &p, const VelBuf &v, void *const F[3], void *const T[3], int32_t n,
                  const Consts &c, const Grid &g, int32_t *cell, int32_t *err, hipStream_t st) {
  k_kick_drift_hash<Real><<<blocks_for(n), kBlock, 0, st>>>(p, v, (const Real *)F[0], (const Real *)F[1],
                                                            (const Real *)F[2], (const Real *)T[0],
                                                            (const Real *)T[1], (const Real *)T[2], n, c, g,
                                                            cell, err);
}

hipError_t launch_kick_drift_hash(int precision, const PosBuf &p, const VelBuf &v, void *const F[3],
                                  void *const T[3], int32_t n, const Consts &c, const Grid &g, int32_t *cell,
                                  int32_t *err, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    kdh_t<double>(p, v, F, T, n, c, g, cell, err, st);
  else
    kdh_t<float>(p, v, F, T, n, c, g, cell, err, st);
  return hipGetLastError();
}

hipError_t launch_reorder(int precision, const PosBuf &src, const VelBuf &vsrc, const PosBuf &dst,
                          const VelBuf &vdst, const int32_t *perm, const int32_t *cell, int32_t *scell,
                          float4 *xyzr, const Grid &g, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    k_reorder<double><<<blocks_for(n), kBlock, 0, st>>>(src, vsrc, dst, vdst, perm, cell, scell, xyzr, g, n);
  else
    k_reorder<float><<<blocks_for(n), kBlock, 0, st>>>(src, vsrc, dst, vdst, perm, cell, scell, xyzr, g, n);
  return hipGetLastError();
}

hipError_t launch_xyzr(const PosBuf &p, float4 *xyzr, const Grid &g, int32_t n, hipStream_t st) {
  if (n > 0) k_xyzr<<<blocks_for(n), kBlock, 0, st>>>(p, xyzr, g, n);
  return hipGetLastError();
}

static hipError_t scan_with_total(const int32_t *in, int32_t *out, int64_t len, const ScanScratch &sc,
                                  hipStream_t st) {
  hipError_t e = scan_exclusive(in, out, len, sc, 0, st);
  if (e != hipSuccess) return e;
  k_scan_total<<<1, 64, 0, st>>>(in, out, len);
  return hipGetLastError();
}

static unsigned pair_blocks() { return 2048; }  // grid-stride over the contacts (count known on device)

hipError_t launch_contacts(const PosBuf &p, const NbrBuf &nb, const PairGen &gen, const PairWork &w,
                           const int32_t *scell, const int32_t *cell_start, const Grid &g, uint32_t wall_mask,
                           int32_t n, const ScanScratch &sc, int32_t *err, hipStream_t st) {
  if (n <= 0) {
    k_fill<<<1, kBlock, 0, st>>>(gen.ofs, 1, 0);
    k_fill<<<1, kBlock, 0, st>>>(w.bofs, 1, 0);
    return hipGetLastError();
  }
  k_detect<<<blocks_for(n), kBlock, 0, st>>>(p, nb, scell, cell_start, g, wall_mask, n, err);
  hipError_t e = scan_with_total(nb.cnt, gen.ofs, n, sc, st);
  if (e != hipSuccess) return e;
  k_fill<<<blocks_for(n), kBlock, 0, st>>>(w.bcnt, n, 0);
  k_pairs<<<blocks_for(n), kBlock, 0, st>>>(nb, p, gen, w, n, err);
  if ((e = scan_with_total(w.bcnt, w.bofs, n, sc, st)) != hipSuccess) return e;
  k_bwd<<<pair_blocks(), kBlock, 0, st>>>(gen, w, n);
  return hipGetLastError();
}

template <typename Real>
static void forces_t(const PairArgs &a, hipStream_t st) {
  switch (a.c.law) {
    case DEM_LAW_HERTZ:
      k_pair_force<Real, DEM_LAW_HERTZ><<<pair_blocks(), kBlock, 0, st>>>(a);
      break;
    case DEM_LAW_SIMPLE:
      k_pair_force<Real, DEM_LAW_SIMPLE><<<pair_blocks(), kBlock, 0, st>>>(a);
      break;
    default:
      k_pair_force<Real, DEM_LAW_LINEAR><<<pair_blocks(), kBlock, 0, st>>>(a);
      break;
  }
  k_gather<Real><<<blocks_for(a.n), kBlock, 0, st>>>(a);
}

hipError_t launch_forces(int precision, const PairArgs &a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    forces_t<double>(a, st);
  else
    forces_t<float>(a, st);
  return hipGetLastError();
}

hipError_t launch_diag_reduce(int precision, const PosBuf &p, const VelBuf &v, const DiagBuf &d, int32_t n,
                              const Consts &c, const Grid &g, hipStream_t st) {
  const int nb = diag_blocks(n);
  if (precision == DEM_PREC_FP64)
    k_diag_partial<double><<<nb, kBlock, 0, st>>>(p, v, d, n, c, g);
  else
    k_diag_partial<float><<<nb, kBlock, 0, st>>>(p, v, d, n, c, g);
  k_diag_final<<<1, kBlock, 0, st>>>(d, nb);
  return hipGetLastError();
}

}  // namespace dem
