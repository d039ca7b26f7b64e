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
//                exactly in FP64; hits go to the particle's own forward list
//                (ascending, no atomics) and to the partner's backward list
//   Steps 7-8    k_force: one lane per sorted particle walks its compact
//                contact list in ascending partner slot, evaluates the contact
//                law (Eqs. 2-10, or Eq. 1) and the walls, sums in that fixed
//                order (no atomics), updates the tangential history and applies
//                the closing half kick
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
__global__ __launch_bounds__(kBlock) void k_kick(PosBuf p, VelBuf vb, const Real *__restrict__ Fx,
                                                 const Real *__restrict__ Fy, const Real *__restrict__ Fz,
                                                 const Real *__restrict__ Tx, const Real *__restrict__ Ty,
                                                 const Real *__restrict__ Tz, int32_t n, Consts c) {
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
}

// --------------------------------------------------------------------------
// Step 3: counting sort by cell, then a canonical order (by id) inside cells

__global__ __launch_bounds__(kBlock) void k_fill(int32_t *a, int64_t len, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < len) a[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_count(const int32_t *__restrict__ cell, int32_t *__restrict__ rank,
                                                  int32_t *counts, int32_t n) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  rank[i] = atomicAdd(&counts[cell[i]], 1);
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
// partner found this way has a higher slot, so the forward list comes out
// ascending without atomics.

constexpr int kSurv = 16;  // LDS survivor slots per lane

// exact FP64 decision on one prefilter survivor, and its recording: the
// particle's own forward list (in order) and the partner's backward list
__device__ __forceinline__ void exact_and_record(const NbrBuf &nb, const PosBuf &pos, int32_t N, int32_t s,
                                                 float ri, double xi, double yi, double zi, int32_t t,
                                                 int32_t &nf, bool &overflow) {
  const double ex = pos.x[t] - xi, ey = pos.y[t] - yi, ez = pos.z[t] - zi;
  const double S = (double)ri + (double)pos.r[t];
  if (!(dist2_exact(ex, ey, ez) < sq_exact(S))) return;
  if (nf < nb.Kd) {
    nb.nb_f[(int64_t)nf * N + s] = t;
  } else {
    overflow = true;
  }
  nf++;
  const int32_t kb = atomicAdd(&nb.cnt_b[t], 1);
  if (kb < nb.Kd) {
    nb.nb_b[(int64_t)kb * N + t] = s;
  } else {
    overflow = true;
  }
}

// Prefilter one slot range; survivors wait in the lane's LDS slots so that
// the rare exact test does not sit inside the candidate loop (where any one
// lane taking it would hold the whole wave).  A lane whose slots fill up
// drains them itself, in order.
__device__ __forceinline__ void prefilter_range(const NbrBuf &nb, const PosBuf &pos, int32_t N, int32_t s,
                                                const float4 p, double xi, double yi, double zi, int32_t beg,
                                                int32_t end, int32_t *surv, int32_t &ns, int32_t &nf,
                                                bool &overflow) {
  for (int32_t t = beg; t < end; t++) {
    const float4 q = nb.xyzr[t];
    const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
    const float sf = p.w + q.w + nb.eps;
    if (dx * dx + dy * dy + dz * dz < sf * sf) {
      if (ns == kSurv) {
        for (int k = 0; k < kSurv; k++)
          exact_and_record(nb, pos, N, s, p.w, xi, yi, zi, surv[k * kBlock], nf, overflow);
        ns = 0;
      }
      surv[ns * kBlock] = t;
      ns++;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_detect(PosBuf pos, NbrBuf nb, const int32_t *__restrict__ scell,
                                                   const int32_t *__restrict__ cell_start, Grid g, int32_t n,
                                                   int32_t *err) {
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
  bool overflow = false;
  // own row: the rest of the own cell and the next cell along x
  const int32_t row0 = (cz * ny + cy) * nx;
  prefilter_range(nb, pos, n, s, p, xi, yi, zi, s + 1, cell_start[row0 + x1 + 1], surv, ns, nf, overflow);
  // next row along y in the same plane
  if (cy + 1 < ny) {
    const int32_t row = (cz * ny + cy + 1) * nx;
    prefilter_range(nb, pos, n, s, p, xi, yi, zi, cell_start[row + x0], cell_start[row + x1 + 1], surv, ns, nf,
                    overflow);
  }
  // the three rows of the next plane along z
  if (cz + 1 < nz) {
    for (int32_t dy = -1; dy <= 1; dy++) {
      const int32_t yy = cy + dy;
      if (yy < 0 || yy >= ny) continue;
      const int32_t row = ((cz + 1) * ny + yy) * nx;
      prefilter_range(nb, pos, n, s, p, xi, yi, zi, cell_start[row + x0], cell_start[row + x1 + 1], surv, ns,
                      nf, overflow);
    }
  }
  // exact tests of the survivors, in slot order
  for (int32_t k = 0; k < ns; k++)
    exact_and_record(nb, pos, n, s, p.w, xi, yi, zi, surv[k * kBlock], nf, overflow);
  nb.cnt_f[s] = nf;
  if (overflow) raise_err(err, ERR_OVERFLOW);
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
          const int32_t u = L[i], w = L[l];
          const bool sw = up ? (u > w) : (u < w);
          L[i] = sw ? w : u;
          L[l] = sw ? u : w;
        }
      }
    }
  }
}

template <int M>
__device__ __forceinline__ void sort_small(int32_t *list, int64_t stride, int32_t cnt) {
  int32_t L[M];
#pragma unroll
  for (int i = 0; i < M; i++) L[i] = i < cnt ? list[i * stride] : INT32_MAX;
  bitonic_sort<M>(L);
#pragma unroll
  for (int i = 0; i < M; i++)
    if (i < cnt) list[i * stride] = L[i];
}

// ascending order of a particle's backward list (entries arrive by atomics)
__device__ __forceinline__ void sort_list(int32_t *list, int64_t stride, int32_t cnt) {
  if (cnt <= 1) return;
  if (cnt <= 4) {
    sort_small<4>(list, stride, cnt);
  } else if (cnt <= 8) {
    sort_small<8>(list, stride, cnt);
  } else if (cnt <= 16) {
    sort_small<16>(list, stride, cnt);
  } else {
    for (int32_t k = 1; k < cnt; k++) {
      const int32_t v = list[k * stride];
      int32_t j = k - 1;
      while (j >= 0 && list[j * stride] > v) {
        list[(j + 1) * stride] = list[j * stride];
        j--;
      }
      list[(j + 1) * stride] = v;
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

// history lookup: the entry with partner `key` in row `row`, or zero
template <typename Real>
__device__ __forceinline__ void hist_find(const HistBuf &hb, int32_t K, int32_t N, int32_t row, int32_t key,
                                          Real h[3]) {
  h[0] = h[1] = h[2] = 0;
  const int32_t cnt = hb.cnt[row];
  const Real *d = (const Real *)hb.d;
  for (int32_t k = 0; k < cnt; k++) {
    if (hb.partner[(int64_t)k * N + row] == key) {
#pragma unroll
      for (int q = 0; q < 3; q++) h[q] = d[((int64_t)q * K + k) * N + row];
      break;
    }
  }
}

template <typename Real, int LAW>
__global__ __launch_bounds__(kBlock) void k_force(ForceArgs a) {
  const int32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= a.n) return;
  const int32_t N = a.n;
  const Consts &c = a.c;
  const Real *VI[3] = {(const Real *)a.vel_in.v[0], (const Real *)a.vel_in.v[1], (const Real *)a.vel_in.v[2]};
  const Real *WI[3] = {(const Real *)a.vel_in.w[0], (const Real *)a.vel_in.w[1], (const Real *)a.vel_in.w[2]};

  const double xi = a.pos.x[s], yi = a.pos.y[s], zi = a.pos.z[s];
  const float rif = a.pos.r[s];
  const double rid = (double)rif;
  const Real ri = (Real)rif;
  const int32_t idi = a.pos.id[s];
  const Real vi[3] = {VI[0][s], VI[1][s], VI[2][s]};
  const Real wi[3] = {WI[0][s], WI[1][s], WI[2][s]};
  const Real mi = mass_of<Real>(c, ri);
  const bool old_perm = (a.mode & MODE_OLD_PERM) != 0;
  const bool write_hist =
      (a.mode & MODE_WRITE_HIST) != 0 && (LAW != DEM_LAW_SIMPLE || (a.mode & MODE_LIST) != 0);
  const bool diag = (a.mode & MODE_DIAG) != 0;
  const int32_t row_i = old_perm ? a.perm[s] : s;

  Real F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  int32_t nnew = 0;
  bool overflow = false;
  double e_el = 0.0, dmax = 0.0;
  int32_t npair = 0, nwall = 0;
  Real *hd = (Real *)a.hnew.d;

  // contact partners in ascending slot: the backward list (lower slots,
  // sorted here) then the forward list (higher slots, ascending)
  const int32_t Kd = a.nbr.Kd;
  const int32_t nbk = min(a.nbr.cnt_b[s], Kd), nfk = min(a.nbr.cnt_f[s], Kd);
  sort_list(a.nbr.nb_b + s, N, nbk);
  for (int32_t k = 0; k < nbk + nfk; k++) {
    const int32_t t = k < nbk ? a.nbr.nb_b[(int64_t)k * N + s] : a.nbr.nb_f[(int64_t)(k - nbk) * N + s];
    const double dx = a.pos.x[t] - xi, dy_ = a.pos.y[t] - yi, dz_ = a.pos.z[t] - zi;
    const double d2 = dist2_exact(dx, dy_, dz_);
    const double S = rid + (double)a.pos.r[t];
    {
        // a contact: evaluate it in the canonical orientation (lower id first)
        // so that both particles compute bit-identical values
        const int32_t idj = a.pos.id[t];
        const bool low = idi < idj;
        const Real rj = (Real)a.pos.r[t];
        const Real vj[3] = {VI[0][t], VI[1][t], VI[2][t]};
        const Real wj[3] = {WI[0][t], WI[1][t], WI[2][t]};
        const Real mj = mass_of<Real>(c, rj);
        const Real ra = low ? ri : rj, rb = low ? rj : ri;
        const Real ma = low ? mi : mj, mb = low ? mj : mi;
        const double ex = low ? dx : -dx, ey = low ? dy_ : -dy_, ez = low ? dz_ : -dz_;
        const Real dd = sqrt((Real)d2);
        const Real invd = (Real)1 / dd;
        const Real n[3] = {(Real)ex * invd, (Real)ey * invd, (Real)ez * invd};
        const Real delta = (Real)(sq_exact(S) - d2) / ((Real)S + dd);
        const Real R = ra * rb / (ra + rb);
        const Real M = ma * mb / (ma + mb);
        Real v[3], spin[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
          const Real va = low ? vi[q] : vj[q], vb = low ? vj[q] : vi[q];
          const Real wa = low ? wi[q] : wj[q], wb = low ? wj[q] : wi[q];
          v[q] = va - vb;
          spin[q] = ra * wa + rb * wb;
        }
        Real h[3] = {0, 0, 0};
        if (LAW != DEM_LAW_SIMPLE) {
          const int32_t hrow = low ? row_i : (old_perm ? a.perm[t] : t);
          hist_find<Real>(a.hold, a.K, N, hrow, low ? idj : idi, h);
        }
        LawOut<Real> o;
        contact_law<Real, LAW>(c, n, delta, R, M, v, spin, h, o);
        const Real sg = low ? (Real)1 : (Real)-1;
        const Real nxft[3] = {n[1] * o.Ft[2] - n[2] * o.Ft[1], n[2] * o.Ft[0] - n[0] * o.Ft[2],
                              n[0] * o.Ft[1] - n[1] * o.Ft[0]};
#pragma unroll
        for (int q = 0; q < 3; q++) {
          F[q] += sg * o.F[q];
          T[q] += ri * nxft[q];  // Eq. 3; same sign on both bodies
        }
        if (low) {
          if (write_hist) {
            if (nnew < a.K) {
              a.hnew.partner[(int64_t)nnew * N + s] = idj;
#pragma unroll
              for (int q = 0; q < 3; q++) hd[((int64_t)q * a.K + nnew) * N + s] = o.dtn[q];
              nnew++;
            } else {
              overflow = true;
            }
          }
          if (diag) {
            e_el += elastic_energy<Real, LAW>(c, delta, R, o, h);
            npair++;
            dmax = fmax(dmax, (double)delta);
          }
        }
    }
  }

  // Step 8: walls, particles of infinite radius
  if (c.wall_mask) {
    const double pos[3] = {xi, yi, zi};
    for (int w = 0; w < 6; w++) {
      if (!((c.wall_mask >> w) & 1)) continue;
      const int ax = w >> 1;
      const double gap = (w & 1) ? (a.grid.hi[ax] - pos[ax]) : (pos[ax] - a.grid.lo[ax]);
      if (!(gap < rid)) continue;
      Real n[3] = {0, 0, 0};
      n[ax] = (w & 1) ? (Real)1 : (Real)-1;
      const Real delta = (Real)(rid - gap);
      Real spin[3];
#pragma unroll
      for (int k = 0; k < 3; k++) spin[k] = ri * wi[k];
      Real h[3] = {0, 0, 0};
      if (LAW != DEM_LAW_SIMPLE) hist_find<Real>(a.hold, a.K, N, row_i, -1 - w, h);
      LawOut<Real> o;
      contact_law<Real, LAW>(c, n, delta, ri, mi, vi, spin, h, o);
      const Real nxft[3] = {n[1] * o.Ft[2] - n[2] * o.Ft[1], n[2] * o.Ft[0] - n[0] * o.Ft[2],
                            n[0] * o.Ft[1] - n[1] * o.Ft[0]};
#pragma unroll
      for (int k = 0; k < 3; k++) {
        F[k] += o.F[k];
        T[k] += ri * nxft[k];
      }
      if (write_hist) {
        if (nnew < a.K) {
          a.hnew.partner[(int64_t)nnew * N + s] = -1 - w;
#pragma unroll
          for (int q = 0; q < 3; q++) hd[((int64_t)q * a.K + nnew) * N + s] = o.dtn[q];
          nnew++;
        } else {
          overflow = true;
        }
      }
      if (diag) {
        e_el += elastic_energy<Real, LAW>(c, delta, ri, o, h);
        nwall++;
        dmax = fmax(dmax, (double)delta);
      }
    }
  }

  if (!(isfinite((double)F[0]) && isfinite((double)F[1]) && isfinite((double)F[2]) &&
        isfinite((double)T[0]) && isfinite((double)T[1]) && isfinite((double)T[2])))
    raise_err(a.err, ERR_NONFINITE);
  if (overflow) raise_err(a.err, ERR_OVERFLOW);
  if (write_hist) a.hnew.cnt[s] = nnew;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    ((Real *)a.F[k])[s] = F[k];
    ((Real *)a.T[k])[s] = T[k];
  }
  if (a.mode & MODE_KICK) {
    Real v[3] = {vi[0], vi[1], vi[2]}, w[3] = {wi[0], wi[1], wi[2]};
    const Real I = (Real)0.4 * mi * ri * ri;
    half_kick<Real>(c, mi, I, F, T, v, w);
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

hipError_t launch_kick(int precision, const PosBuf &p, const VelBuf &v, void *const F[3], void *const T[3],
                       int32_t n, const Consts &c, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    k_kick<double><<<blocks_for(n), kBlock, 0, st>>>(p, v, (const double *)F[0], (const double *)F[1],
                                                     (const double *)F[2], (const double *)T[0],
                                                     (const double *)T[1], (const double *)T[2], n, c);
  else
    k_kick<float><<<blocks_for(n), kBlock, 0, st>>>(p, v, (const float *)F[0], (const float *)F[1],
                                                    (const float *)F[2], (const float *)T[0],
                                                    (const float *)T[1], (const float *)T[2], n, c);
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

hipError_t launch_detect(const PosBuf &p, const NbrBuf &nb, const int32_t *scell, const int32_t *cell_start,
                         const Grid &g, int32_t n, int32_t *err, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill<<<blocks_for(n), kBlock, 0, st>>>(nb.cnt_b, n, 0);
  k_detect<<<blocks_for(n), kBlock, 0, st>>>(p, nb, scell, cell_start, g, n, err);
  return hipGetLastError();
}

template <typename Real>
static void force_t(const ForceArgs &a, hipStream_t st) {
  switch (a.c.law) {
    case DEM_LAW_HERTZ:
      k_force<Real, DEM_LAW_HERTZ><<<blocks_for(a.n), kBlock, 0, st>>>(a);
      break;
    case DEM_LAW_SIMPLE:
      k_force<Real, DEM_LAW_SIMPLE><<<blocks_for(a.n), kBlock, 0, st>>>(a);
      break;
    default:
      k_force<Real, DEM_LAW_LINEAR><<<blocks_for(a.n), kBlock, 0, st>>>(a);
      break;
  }
}

hipError_t launch_force(int precision, const ForceArgs &a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (precision == DEM_PREC_FP64)
    force_t<double>(a, st);
  else
    force_t<float>(a, st);
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
