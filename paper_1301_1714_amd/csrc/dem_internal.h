// dem_internal.h -- device data layout and kernel launchers of libdem.so.
//
// One engine holds S >= 1 independent systems.  Their particles occupy fixed,
// consecutive slot ranges [p0, p0 + n) and their cells consecutive global
// cell ranges [c0, c0 + ncell); the cell sort keeps every particle inside its
// system's slot range, so the particle -> system map never changes.
//
// Layout in HBM (structure of arrays, per-particle arrays indexed by the
// sorted slot of the last cell sort, Sec. 4.1 / Step 4):
//   pos[2]   x, y, z (FP64), r (FP32), id (int32; unique over the engine)
//   vel[2]   vx, vy, vz, wx, wy, wz (Real)
//   F, T     contact force / torque of the last evaluation (Real)
//   cell     global cell of the pre-sort order; rank, perm (new -> old slot)
//   scell    global cell of each sorted slot; cell_start[ncell_total + 1]
//   psys     system of each slot; bsys/bfirst: system and first slot of each
//            kernel block (blocks never straddle two systems)
//   nbr      detection input and output: xyzr (FP32 copy of x - lo and r)
//            and xq (8-byte fixed-point copy, the direct sweep's candidate
//            records), and, per particle, its contacts with higher slots in
//            ascending order followed by its walls (-1 - w)
//   pst      the law's inputs per particle, packed (PState<Real>), with the
//            previous slot and committed history segment of each slot
//   tiles    detection work items: (system, row, first cell, last cell) of
//            the LDS-tiled shape; runs: the same for the wave shape
//   gen[2]   two generations of the compact contact array, CSR by owner slot
//            (the lower slot of a pair; the particle for a wall): ofs[N + 1],
//            per contact the owner s and partner t (slot or -1 - w), and one
//            Real4 entry of the tangential-history table: delta_t as seen
//            from the owner in x, y, z and the key (t, its bits) in w, so
//            that one load brings both.  One generation holds the committed
//            history, the other is built for the new positions.
//   work     per-contact force on the owner and n x F_t (6 Real), and the
//            backward lists (contacts of each particle as the partner)
// Real is double (DEM_PREC_FP64) or float (DEM_PREC_MIXED).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dem.h"

namespace dem {

enum ErrBits : int32_t { ERR_DOMAIN = 1, ERR_OVERFLOW = 2, ERR_NONFINITE = 4 };

// contact-evaluation modes
enum ModeBits : int32_t {
  MODE_WRITE_HIST = 1,  // write the new tangential displacements
  MODE_KICK = 2,        // a time step: closing half kick (active systems only)
  MODE_DIAG = 4,        // per-particle elastic energy / contact counts / max overlap
  MODE_OLD_PERM = 8     // committed history is in the pre-sort slot order (the records say where)
};

constexpr int32_t kBlock = 256;
constexpr int32_t kListCap = 64;  // detection: contacts per particle (higher partners + walls)
// contact-list offsets are int32: n * kListCap must stay below 2^31
constexpr int64_t kMaxParticles = INT32_MAX / kListCap;
constexpr int32_t kBwdCap = 32;   // contacts per particle with lower partners
constexpr int32_t kMaxTile = 32;  // cells along x per detection tile
constexpr int32_t kRunCells = 8;  // cells along x per wave of the wave-per-cell-run detection
constexpr int32_t kMaxReach = 2;  // largest cell divisor

struct Grid {
  double lo[3], hi[3];
  double sc[3];  // cells per unit length: n_a / (hi_a - lo_a)
  int32_t nc[3];
  int32_t c0;     // first global cell of the system
  int32_t ncell;  // cells of the system
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

struct SysInfo {
  Grid g;
  Consts c;
  int32_t p0, n;  // slot range
  float eps;      // detection prefilter margin
  float rmax;     // largest radius (FP32), bounds the contact distance
  int32_t tile;   // detection: cells per tile (0: direct sweep, -1: wave per cell run)
  int32_t reach;  // cells swept on each side of a particle's own (the cell divisor)
};

// Step control on the device, so that one captured step can be replayed:
// system k is active while step < left[k]; a step after which it stays
// active also runs the next step's opening kick, drift and hash.
struct StepCtl {
  int32_t *step;  // [1] steps done in the current call
  int32_t *left;  // [S] steps requested for each system in the current call
};

struct PosBuf {
  double *x, *y, *z;
  float *r;
  int32_t *id;
};

struct VelBuf {
  void *v[3], *w[3];
};

// The state the contact law reads, packed per particle so that a partner
// costs one or two cache lines instead of one per array.  In a time step it
// also carries where the particle's committed tangential history is: its
// previous slot (low kPrevBits bits of hp) and the count (high bits) and
// first index (hb) of the contacts it owned there.
constexpr int kPrevBits = 25;
static_assert(kMaxParticles <= (1 << kPrevBits), "previous slot must fit in kPrevBits bits");
static_assert(kListCap < (1 << (32 - kPrevBits)), "history count must fit above the previous slot");
template <typename Real>
struct alignas(16) PState {
  double x, y, z;
  Real v[3], w[3];
  float r;
  int32_t id;
  uint32_t hp;  // previous slot | owned history count << kPrevBits
  int32_t hb;   // first committed history entry of the previous slot
};

struct NbrBuf {
  float4 *xyzr;   // [N] (x - lo, y - lo, z - lo, r), FP32; written only while a system uses tiles or waves
  uint2 *xq;      // [N] x, y, z in cell units modulo 8 cells (1/8192 cell, 16 bits each), r in rmax/65535 rounded up
  int32_t *fcnt;  // [N] entries of nb (clamped to kListCap)
  int32_t *nb;    // [kListCap][N]
  void *pst;      // [N] PState<Real> of the current slots
};

struct PairGen {
  int32_t *ofs;  // [N + 1]
  int32_t *s;    // [Pcap] owner slot
  int32_t *t;    // [Pcap] partner slot or -1 - w
  void *ent;     // [Pcap] Real4: delta_t (x, y, z), key bits (w)
};

struct PairWork {
  void *pf;        // [6 Pcap] Real: force on the owner, then n x F_t
  double *pe;      // [Pcap] elastic energy (diagnostics)
  double *pd;      // [Pcap] overlap (diagnostics)
  int32_t *bcnt;   // [N] contacts of each particle as the partner
  int32_t *bwd;    // [kBwdCap][N] their indices, in arrival order
};

struct DiagBuf {
  double *e_el;     // [N] elastic energy of the contacts a particle owns
  int32_t *npair;   // [N]
  int32_t *nwall;   // [N]
  double *dmax;     // [N]
  double *partial;  // [blocks][10]
  double *out;      // [S][10]
};

// what every per-particle kernel needs to find its system
struct Layout {
  const SysInfo *tab;     // [S]
  const int32_t *psys;    // [N]
  const int32_t *bsys;    // [nblocks]
  const int32_t *bfirst;  // [nblocks]
  const int4 *tiles;      // [ntiles] (system, y + ny z, first cell x, last cell x)
  const int4 *runs;       // [nruns] the same for the wave-per-cell-run detection
  int32_t nblocks;
  int32_t ntiles;
  int32_t nruns;
  int32_t ndirect;  // systems swept by the direct detection kernel with reach 1
  int32_t ndirect2; // and with reach 2
  int32_t n;
  int32_t S;
};

struct PairArgs {
  Layout L;
  StepCtl ctl;
  PosBuf pos;            // current positions
  PosBuf pos_out;        // time steps: positions after the step (drifted for the next one)
  VelBuf vel_in, vel_out;
  NbrBuf nb;             // packed state and history index of the current slots
  PairGen cur, old;      // cur: contacts of the current positions; old: committed history
  PairWork w;
  int64_t cap;           // contacts a table holds
  void *F[3], *T[3];
  DiagBuf diag;
  int32_t *cell;         // cells for the next sort (drifted positions, or unchanged ones)
  const int32_t *scell;  // cells of the current slots
  int32_t mode;
  int32_t law;
  int32_t *err;
};

struct ScanScratch {
  int32_t *level[4];  // block sums per level
  int64_t len[4];
  int nlevels;
};

// launchers (dem_kernels.hip); all enqueue on `st` and return hipError_t
hipError_t launch_hash(const Layout &L, const PosBuf &p, int32_t *cell, int32_t *err, hipStream_t st);
hipError_t launch_kick_drift_hash(int precision, const Layout &L, const StepCtl &ctl, const PosBuf &p,
                                  const VelBuf &v, void *const F[3], void *const T[3], const int32_t *scell,
                                  int32_t *cell, int32_t *err, hipStream_t st);
hipError_t launch_sort(const int32_t *cell, const int32_t *id_old, int32_t n, int64_t ncell, int32_t *counts,
                       int32_t *rank, int32_t *cell_start, int32_t *perm, const ScanScratch &sc, hipStream_t st);
// Step 4 into the packed records nb.pst (and, with soa, into dst / vdst as
// well; a time step leaves that to its gather); old_ofs: offsets of the
// committed history, whose segments are recorded in the records (nullptr:
// none)
hipError_t launch_reorder(int precision, const Layout &L, const PosBuf &src, const VelBuf &vsrc, const PosBuf &dst,
                          const VelBuf &vdst, bool soa, const int32_t *perm, const int32_t *cell, int32_t *scell,
                          const NbrBuf &nb, const int32_t *old_ofs, hipStream_t st);
hipError_t launch_xyzr(const Layout &L, const PosBuf &p, const NbrBuf &nb, hipStream_t st);
// nb.pst from the current buffers (before a force evaluation outside a step)
hipError_t launch_pack(int precision, const Layout &L, const PosBuf &p, const VelBuf &v, const NbrBuf &nb,
                       hipStream_t st);
// Steps 5-6: detection (all systems, or with ctl only the active ones; the
// others keep their lists), then the compact contact array of `gen` and its
// backward index
hipError_t launch_detect(int precision, const Layout &L, const StepCtl *ctl, const NbrBuf &nb,
                         const int32_t *scell, const int32_t *cell_start, int32_t *err, hipStream_t st);
// (write_keys: also write the history keys into the entries; a time step
// whose law keeps history leaves that to the law pass)
hipError_t launch_list(int precision, const Layout &L, const NbrBuf &nb, const PairGen &gen, const PairWork &w,
                       int64_t cap, bool write_keys, const ScanScratch &sc, int32_t *err, hipStream_t st);
// Steps 7-8: the law once per contact, then per-particle sums and (in a time
// step) the kicks
hipError_t launch_pair_force(int precision, const PairArgs &a, hipStream_t st);
hipError_t launch_gather(int precision, const PairArgs &a, hipStream_t st);
hipError_t launch_step_end(const StepCtl &ctl, hipStream_t st);
hipError_t launch_diag_reduce(int precision, const Layout &L, const PosBuf &p, const VelBuf &v, const DiagBuf &d,
                              hipStream_t st);
hipError_t launch_fill(int32_t *a, int64_t len, int32_t value, hipStream_t st);
int64_t scan_scratch_len(int64_t n, int64_t *lens, int *nlevels);

}  // namespace dem
