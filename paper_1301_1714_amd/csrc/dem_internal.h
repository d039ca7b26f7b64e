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
//            records); per particle the contacts it owns (partners with
//            higher slots in ascending order, then its walls as -1 - w),
//            K of them at most (the system's contacts_per_particle), stored
//            k-major: entry k of slot s at [k * N + s]
//   pst      the law's inputs per particle, packed (PState<Real>), with the
//            previous slot and committed history count of each slot
//   tiles    detection work items: (system, row, first cell, last cell) of
//            the LDS-tiled shape; runs: the same for the wave shape
//   hist[2]  two generations of the tangential-history table: per slot its
//            count and the index of its first entry, and one Real4 entry per
//            owned contact: delta_t as seen from the owner in x, y, z and the
//            key (partner slot or -1 - w, its bits) in w, so that one load
//            brings both.  One generation holds the committed history, the
//            other is written for the new positions.
//   work     per owned contact: force on the owner and n x F_t (6 Real), and
//            the backward lists (contacts of each particle as the partner,
//            each as the index of its contact record)
// Per-contact arrays (history entries, force records) keep the contacts of
// one kernel block together: block b owns kBlock * K entries from
// cbase(b, K), and contact k of slot s sits at cbase(b, K) + off(s) + k,
// off(s) the exclusive prefix of the owned counts over the block's slots in
// order.  A wave's contacts are then one contiguous run (its stores coalesce)
// and a particle's history entries are adjacent (one line per lookup).
// Real is double (DEM_PREC_FP64) or float (DEM_PREC_MIXED).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dem.h"

namespace dem {

enum ErrBits : int32_t { ERR_DOMAIN = 1, ERR_OVERFLOW = 2, ERR_NONFINITE = 4 };

// A law template argument is the dem_law plus kLawTerms when the optional
// contact terms are compiled in (engines where some system uses them) and
// plus kLawFull when the material-pair tables and the diagnostics are (an
// engine where some system may have a table, or a diagnostics pass).  The
// lean form needs fewer registers, so more waves share each SIMD.
constexpr int kLawTerms = 4;
constexpr int kLawFull = 8;

// contact-evaluation modes
enum ModeBits : int32_t {
  MODE_WRITE_HIST = 1,  // write the new tangential displacements
  MODE_KICK = 2,        // a time step: closing half kick (active systems only)
  MODE_DIAG = 4,        // per-particle elastic energy / contact counts / max overlap
  MODE_OLD_PERM = 8     // committed history is in the pre-sort slot order (the records say where)
};

constexpr int32_t kBlock = 256;
constexpr int32_t kBackCap = 1024;  // backward contacts filed per kernel block (more: found by a scan)
constexpr int32_t kListCap = 64;  // largest per-particle capacity of owned contacts (higher partners + walls)
// contact indices k * N + s are int32: n * kListCap must stay below 2^31
constexpr int64_t kMaxParticles = INT32_MAX / kListCap;
// first entry of kernel block b's contacts (see the layout above)
__host__ __device__ inline int64_t cbase(int32_t b, int32_t K) { return (int64_t)b * kBlock * K; }
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
  uint32_t terms;  // DEM_TERM_* bits of the system
  double cohesion, rolling_mu;
};

// Contact constants of one pair of materials (Sec. 3: the C_kn, C_kt and
// alpha of Eqs. 8-10 carry the indices of the two bodies in contact; so does
// the Coulomb coefficient of Eq. 5 here)
struct PairK {
  double kn, kt, alpha, mu;
};
constexpr int32_t kMaxMaterials = 16;

// a finite wall (dem_plate): the rectangle x[axis] = at, lo..hi on the
// axes (axis + 1) % 3 and (axis + 2) % 3
struct Plate {
  int32_t axis, pad;
  double at;
  double lo[2], hi[2];
};
constexpr int32_t kMaxPlates = DEM_MAX_PLATES;

struct SysInfo {
  Grid g;
  Consts c;
  int32_t nplates;             // plates, walls 6 .. 5 + nplates
  Plate plates[kMaxPlates];
  int32_t ntypes;     // materials of the system's table (0: one material, the constants in c)
  int32_t mat0;       // its first entry in the engine's table: (t, u) at mat0 + t * ntypes + u
  int32_t wall_type;  // material of the walls
  int32_t p0, n;  // slot range
  float eps;      // detection prefilter margin
  float rmax;     // largest radius (FP32), bounds the contact distance
  int32_t tile;   // detection: cells per tile (0: direct sweep, -1: wave per cell run)
  int32_t reach;  // cells swept on each side of a particle's own (the cell divisor)
  int32_t kcap;   // owned contacts per particle at most (contacts_per_particle)
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
  int32_t *mt;  // material of each slot (nullptr: no system of the engine has a material table)
};

struct VelBuf {
  void *v[3], *w[3];
};

// The state the contact law reads, packed per particle so that a partner
// costs one or two cache lines instead of one per array.  In a time step it
// also carries where the particle's committed tangential history is: its
// previous slot (low kPrevBits bits of hp), the number of contacts it owned
// there (high bits) and the index of the first of their entries (hq).  The
// particle's material rides in the bits of the id above kMtShift.
constexpr int kPrevBits = 25;
constexpr int kMtShift = 25;
constexpr int32_t kIdMask = (1 << kMtShift) - 1;
static_assert(kMaxParticles <= (1 << kMtShift), "ids must fit below the material bits");
static_assert(kMaxParticles <= (1 << kPrevBits), "previous slot must fit in kPrevBits bits");
static_assert(kListCap < (1 << (32 - kPrevBits)), "history count must fit above the previous slot");
template <typename Real>
struct alignas(16) PState {
  double x, y, z;
  Real v[3], w[3];
  float r;
  int32_t id;
  uint32_t hp;  // previous slot | owned history count << kPrevBits
  int32_t hq;   // index of the first committed history entry of the previous slot
};

struct NbrBuf {
  float4 *xyzr;   // [N] (x - lo, y - lo, z - lo, r), FP32; written only while a system uses tiles or waves
  uint2 *xq;      // [N] x, y, z in cell units modulo 8 cells (1/8192 cell, 16 bits each), r in rmax/65535 rounded up
  int32_t *fcnt;  // [N] owned contacts (clamped to the capacity K)
  int32_t *nb;    // [K][N] their partners
  void *pst;      // [N] PState<Real> of the current slots
  int32_t K;      // owned contacts per particle at most (largest contacts_per_particle of the engine)
};

// one generation of the tangential-history table
struct HistGen {
  int32_t *cnt;    // [N] entries of each slot
  int32_t *start;  // [N] index of each slot's first entry
  void *ent;       // [blocks * kBlock * K] Real4: delta_t (x, y, z), key bits (w)
};

struct PairWork {
  void *pf;        // per contact 3 x Real2: force on the owner, then n x F_t
  void *pc;        // per contact Real4: the couple of the optional terms on the owner (engines with terms only)
  double *pe;      // per contact elastic energy (diagnostics)
  double *pd;      // per contact overlap (diagnostics)
  int32_t *qs;     // [N] index of each slot's first owned contact
  int2 *back;      // [nblocks][kBackCap] per kernel block, the contacts whose partner is
                   // one of its slots: (contact index, partner slot), in arrival order
  int32_t *nback;  // [nblocks] their number (zero between evaluations)
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
  const PairK *mat;       // material-pair tables of the systems that have one
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
  NbrBuf nb;             // packed state and history index of the current slots; owned contacts
  HistGen cur, old;      // cur: history written for the current positions; old: committed history
  PairWork w;
  void *F[3], *T[3];
  DiagBuf diag;
  int32_t *cell;         // cells for the next sort (drifted positions, or unchanged ones)
  const int32_t *scell;  // cells of the current slots
  const int32_t *cell_start;  // their cells' first slots
  int32_t mode;
  int32_t law;
  int32_t terms;         // some system of the engine has optional contact terms (dem_params.terms)
  int32_t mats;          // some system of the engine may have a material-pair table (max_materials > 0)
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
// Step 3.  cell_old: the cells of the input slots before this sort (the
// previous sort's order), nullptr for a first sort; flags: one byte per cell,
// zero between sorts (cells whose order inside must be set again)
hipError_t launch_sort(const int32_t *cell, const int32_t *id_old, const int32_t *cell_old, int32_t n,
                       int64_t ncell, int32_t *counts, int32_t *rank, int32_t *cell_start, int32_t *perm,
                       uint8_t *flags, const ScanScratch &sc, hipStream_t st);
// Step 4 into the packed records nb.pst (and, with soa, into dst / vdst as
// well; a time step leaves that to its gather); old: the committed history,
// whose count and first entry per previous slot are recorded in the records
// with the previous slots (nullptr: none)
hipError_t launch_reorder(int precision, const Layout &L, const PosBuf &src, const VelBuf &vsrc, const PosBuf &dst,
                          const VelBuf &vdst, bool soa, const int32_t *perm, const int32_t *cell, int32_t *scell,
                          const NbrBuf &nb, const HistGen *old, hipStream_t st);
hipError_t launch_xyzr(const Layout &L, const PosBuf &p, const NbrBuf &nb, hipStream_t st);
// nb.pst from the current buffers (before a force evaluation outside a step)
hipError_t launch_pack(int precision, const Layout &L, const PosBuf &p, const VelBuf &v, const NbrBuf &nb,
                       hipStream_t st);
// Steps 5-8: detection of the owned contacts (all systems, or with ctl only
// the active ones; the others keep their lists).  With `a` the contact law
// follows in the same pass (one lane per contact, compacted per wave) for the
// systems swept by the direct shape, and in a second pass for the others;
// without it only the lists are built.
hipError_t launch_contacts(int precision, const Layout &L, const StepCtl *ctl, const NbrBuf &nb,
                           const int32_t *scell, const int32_t *cell_start, const PairArgs *a, int32_t *err,
                           hipStream_t st, hipEvent_t after_detect);
// per-particle sums and (in a time step) the kicks
hipError_t launch_gather(int precision, const PairArgs &a, hipStream_t st);
hipError_t launch_step_end(const StepCtl &ctl, hipStream_t st);
// largest |v| of each system into vmax[S] (bits of non-negative doubles; zeroed by the caller)
hipError_t launch_max_speed(int precision, const Layout &L, const VelBuf &v, unsigned long long *vmax,
                            hipStream_t st);
hipError_t launch_diag_reduce(int precision, const Layout &L, const PosBuf &p, const VelBuf &v, const DiagBuf &d,
                              hipStream_t st);
hipError_t launch_fill(int32_t *a, int64_t len, int32_t value, hipStream_t st);
int64_t scan_scratch_len(int64_t n, int64_t *lens, int *nlevels);

}  // namespace dem
