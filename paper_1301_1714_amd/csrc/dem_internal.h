// dem_internal.h -- device data layout and kernel launchers of libdem.so.
//
// Layout in HBM (structure of arrays, every array indexed by the sorted slot
// of the last cell sort, Sec. 4.1 / Step 4):
//   pos[2]   x, y, z (FP64), r (FP32), id (int32)          -- double-buffered
//   vel[2]   vx, vy, vz, wx, wy, wz (Real)                   -- double-buffered
//   F, T     contact force / torque of the last evaluation (Real)
//   cell     CM of the pre-sort order; rank, perm (new slot -> old slot)
//   scell    cell of each sorted slot; cell_start[ncell + 1]
//   hist[2]  tangential-history rows, one per slot: cnt, partner[K][N] and
//            delta_t[3][K][N] (Real); a row holds the contacts of its particle
//            with higher-id partners and with walls (partner = -1 - w)
//   nbr      contact lists of the current positions: xyzr (FP32 copy of
//            x - lo and r, the detection prefilter's input), forward partners
//            (higher slots, found by the particle itself, ascending) and
//            backward partners (lower slots, appended by them)
// Real is double (DEM_PREC_FP64) or float (DEM_PREC_MIXED).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dem.h"

namespace dem {

enum ErrBits : int32_t { ERR_DOMAIN = 1, ERR_OVERFLOW = 2, ERR_NONFINITE = 4 };

// force-kernel modes
enum ModeBits : int32_t {
  MODE_WRITE_HIST = 1,  // write the new history rows
  MODE_KICK = 2,        // closing half kick into the other velocity buffer
  MODE_DIAG = 4,        // per-particle elastic energy / contact counts / max overlap
  MODE_OLD_PERM = 8,    // old history rows are found through perm (after a re-sort)
  MODE_LIST = 16        // with MODE_WRITE_HIST: record contacts even for the simple law
};

struct Grid {
  double lo[3], hi[3];
  double sc[3];  // cells per unit length: n_a / (hi_a - lo_a)
  int32_t nc[3];
  int64_t ncell;
};

struct Consts {
  double dt, half_dt;
  double mass_c;  // density * 4/3 * pi
  double alpha, eta_t_ratio;
  double kn, kt, mu;
  double k_sp, k_da, k_sh;
  double g[3];
  uint32_t wall_mask;
  int32_t law;
};

struct PosBuf {
  double *x, *y, *z;
  float *r;
  int32_t *id;
};

struct VelBuf {
  void *v[3], *w[3];
};

struct HistBuf {
  int32_t *cnt;      // [N]
  int32_t *partner;  // [K][N]
  void *d;           // [3][K][N] Real
};

struct NbrBuf {
  float4 *xyzr;    // [N] (x - lo, y - lo, z - lo, r), FP32
  int32_t *cnt_f;  // [N]
  int32_t *nb_f;   // [Kd][N] partner slots > own slot, ascending
  int32_t *cnt_b;  // [N]
  int32_t *nb_b;   // [Kd][N] partner slots < own slot, in arrival order
  int32_t Kd;
  float eps;       // prefilter margin: bounds the FP32 error of |x_j - x_i|
};

struct DiagBuf {
  double *e_el;     // [N] elastic energy of the contacts a particle owns
  int32_t *npair;   // [N]
  int32_t *nwall;   // [N]
  double *dmax;     // [N]
  double *partial;  // [blocks][10]
  double *out;      // [10]
};

struct ForceArgs {
  PosBuf pos;
  NbrBuf nbr;
  VelBuf vel_in, vel_out;
  const int32_t *scell;
  const int32_t *cell_start;
  const int32_t *perm;
  HistBuf hold, hnew;
  void *F[3], *T[3];
  DiagBuf diag;
  int32_t K;
  int32_t n;
  int32_t mode;
  Grid grid;
  Consts c;
  int32_t *err;
};

struct ScanScratch {
  int32_t *level[4];  // block sums per level
  int64_t len[4];
  int nlevels;
};

// launchers (dem_kernels.hip); all enqueue on `st` and return hipError_t
hipError_t launch_hash(const PosBuf &p, int32_t n, const Grid &g, int32_t *cell, int32_t *err, hipStream_t st);
hipError_t launch_kick_drift_hash(int precision, const PosBuf &p, const VelBuf &v, void *const F[3],
                                  void *const T[3], int32_t n, const Consts &c, const Grid &g, int32_t *cell,
                                  int32_t *err, hipStream_t st);
hipError_t launch_kick(int precision, const PosBuf &p, const VelBuf &v, void *const F[3], void *const T[3],
                       int32_t n, const Consts &c, hipStream_t st);
hipError_t launch_sort(const int32_t *cell, const int32_t *id_old, int32_t n, int64_t ncell, int32_t *counts,
                       int32_t *rank, int32_t *cell_start, int32_t *perm, const ScanScratch &sc, hipStream_t st);
hipError_t launch_reorder(int precision, const PosBuf &src, const VelBuf &vsrc, const PosBuf &dst,
                          const VelBuf &vdst, const int32_t *perm, const int32_t *cell, int32_t *scell,
                          float4 *xyzr, const Grid &g, int32_t n, hipStream_t st);
hipError_t launch_xyzr(const PosBuf &p, float4 *xyzr, const Grid &g, int32_t n, hipStream_t st);
hipError_t launch_detect(const PosBuf &p, const NbrBuf &nb, const int32_t *scell, const int32_t *cell_start,
                         const Grid &g, int32_t n, int32_t *err, hipStream_t st);
hipError_t launch_force(int precision, const ForceArgs &a, hipStream_t st);
hipError_t launch_diag_reduce(int precision, const PosBuf &p, const VelBuf &v, const DiagBuf &d, int32_t n,
                              const Consts &c, const Grid &g, hipStream_t st);
int64_t scan_scratch_len(int64_t n, int64_t *lens, int *nlevels);
int diag_blocks(int32_t n);

}  // namespace dem
