// device_types.hpp -- plain structs shared by the host driver and the HIP kernels.
#pragma once

#include <cstdint>

namespace pmg {

constexpr int kMaxLevels = 12;   // MGRIT time levels per instance
// Prefetched triangular-solve limits (512 threads with 4 lanes per row slot, or 1024 with 8): 128 row
// slots per level, up to 64 off-block entries per row and dense diagonal blocks of up to 72 rows.
constexpr int kRowSlots = 128;
constexpr int kOffMax = 64;
// the prefetched triangular solve reads its slot tables through buffer descriptors of this many
// bytes (every table of that path is smaller); an offset at or past it reads zeros
constexpr unsigned kBufBytes = 0x7ffff000u;
constexpr int kDenseMax = 72;
// window mode (work vectors in global memory, latency-bound levels): blocks of up to 128 rows, so
// dense rows of up to 128 entries and half as many dependent levels
constexpr int kDenseWin = 128;
constexpr int kWinBlock = 128;
// words of the triangular solves' LDS block-sum buffer (a level's rows plus the dense rows' reach)
constexpr int kSbufWords = 320;
// LDS staging area of the exact p = 1 solve's dense transforms (doubles)
constexpr int kStageDoubles = 2048;
// largest mesh (elements per direction) whose level-0 steps MGRIT's learned warm start predicts
constexpr int kNetMaxElems = 64;
constexpr int kBandStageMin = 16 * 1024;  // smallest LDS staging area of the band passes (bytes)
// slab tables of the window-mode triangular solves: 8 KB chunks (one 16-byte load per lane of a
// 512-thread workgroup), at most kDch per level, the first slab at value kSlab0 of dfast
constexpr int kChunkBytes = 8192;
constexpr int kDch = 5;  // FP32
template <typename VT>
constexpr int kDchOf = sizeof(VT) == 4 ? kDch : 2 * kDch;
constexpr int kSlab0 = kChunkBytes / 4;
// LDS per workgroup of gfx950 (160 KiB)
constexpr int kLdsBytes = 160 * 1024;
// default row-block size of the triangular solves
constexpr int kWaveBlock = 64;

// per (level, row slot) metadata of the prefetched triangular solve
struct Meta4 {
  int row;   // row (or -1 for an empty slot)
  int bo;    // offset of the row's dense values in dfast (a multiple of 16 bytes)
  int bqc;   // s position of the first dense column (low 16 bits, a multiple of 16 bytes' worth of
             // values) | dense values per lane << 16 (the row holds TG x that many for TG lanes
             // per row, lane g reading 16-byte units g, g + TG, ...)
  int na;    // off-block entries of the row (the rest of its AS-wide row is padding)
};

// level-scheduled blocked triangular solve (see TriSchedule in host_setup.hpp)
struct TriDev {
  int nlev, bs, max_rows, fast;  // fast: the schedule fits the prefetched register path
  // prefetched path: slot tables with addresses computable from (level, row slot, lane)
  int R, AS;                     // row slots per level, off-block row width (ka * lanes per row)
  // window mode (winW > 0, y not in LDS): the off-block columns are slots of an LDS window of the
  // last winW grid lines of winN rows each, line j at slot (j mod winW), so each level reads the
  // lines it couples to from LDS while the solution goes to y in global memory
  int winW, winN;
  // entry 0 of every table is a reserved zero / empty slot
  const Meta4* meta;             // [1 + (nlev + 2) * R]
  const void* dfast;             // dense rows, natural column order, 4 * Meta4::bc values each
  const void* aval;              // [(1 + nlev * R) * AS] off-block values, row 0 = padding
  const int* acol;               // [(1 + nlev * R) * AS] off-block columns minus the zero word's
                                 // index (padding: 0, i.e. the zero word)
  // FP32 window-mode slab tables (dch > 0): level l's dense rows lie contiguous, in row-slot order,
  // in dfast[kSlab0 + l * lsv, + lsv) (lsv = dch x kChunkBytes / 4 values; Meta4::bo stays absolute),
  // and acol16 holds the off-block columns as 16-bit values, lane g's KA of them contiguous at
  // (1 + l * R + r) * AS + g * KA
  int dch, lsv;
  const short* acol16;
  // general path: level-ordered CSR
  const int* lev_ptr;
  const int* row;
  const int* orp;
  const int* oci;
  const void* ov;     // off-block values (V-cycle precision)
  const int* dq0;
  const int* dcnt;
  const int64_t* doff;
  const void* dval;   // dense diagonal-block inverses (V-cycle precision)
};

// a banded 1D factor of a Kronecker product: rows x w values, entry (o, o + lo + d) at [o*w + d]
struct BandDev {
  const double* f64;
  const void* vt;     // V-cycle precision copy
  int rows, w, lo, pad;
};

// one MGRIT time level of one instance: A_l = M + kappa dt_l K and its smoother / coarse data
struct LevelDev {
  double dt, c;        // c = theta kappa dt_l (A_l = M + c K, theta-scheme of Sec. 2)
  double cb;           // cb = (1 - theta) kappa dt_l (B_l = M - cb K applied to the previous point)
  BandDev X1;          // first-direction factor of A_l's first term: Mx + c Kx
  BandDev XB;          // first-direction factor of B_l's first term: Mx - cb Kx (cb != 0 only)
  TriDev L, U;         // ILUT(A_l) factors (slot tables for 4 lanes per row)
  TriDev L8, U8;       // the same factors, slot tables for 8 lanes per row
  const double* tl;    // exact p = 1 solve: Thomas multipliers, node-major [node][mode] (n1 x n1)
  const double* tdinv; //                    inverse pivots, node-major
  const double* htl;   // h-multigrid p = 1 solve: Thomas data of the coarsest h-level, node-major
  const double* htd;
  const double* dgA;   // diag(A_l) (ndof), for Jacobi-preconditioned CG
};

// One h-multigrid W-cycle as the p = 1 solve (Sec. 4, the paragraph after step 5).  h-level 0 is
// the p = 1 space on n elements per direction; each further level halves the mesh while the element
// count is even and above 4.  Operators are Galerkin products R A P with the canonical prolongation
// P and R = P^T, which on these separable geometries keep the form
//   A_k = My_k (x) (Mx_k + c Kx_k) + c Ky_k (x) Mx2_k
// with 1D tridiagonal factors (c = theta kappa dt_l of the MGRIT level).
constexpr int kHmgMax = 12;
struct HmgDev {
  int nh;                        // h-levels (1: the p = 1 problem is solved exactly at once)
  int n1[kHmgMax];               // interior nodes per direction of h-level k
  int64_t off[kHmgMax];          // scratch offset (doubles) of b_k; x_k follows it (k >= 1)
  int64_t words;                 // scratch doubles per workgroup (residual temporary first)
  const double* band[kHmgMax];   // [5][n1][3]: Mx, Kx, Mx2, My, Ky rows (i, i-1), (i, i), (i, i+1)
  const double* Vc;              // coarsest level: generalized eigenvectors of (Ky, My), [iy][k]
};

// A_l = My (x) X1_l + c_l Ky (x) Mx2, M = My (x) Mx, P_1^p = Py (x) Px (second direction slow)
struct InstDev {
  int ndof, n1, ndof1, nlev;
  int nt, nin, p, pad0;
  BandDev Mx, Mx2, My, Ky;   // nin x (2p+1)
  BandDev Kx;                // nin x (2p+1): stiffness factor (the learned guess's explicit increment)
  BandDev Px, Py;            // nin x (p+2): prolongation directions
  BandDev PxT, PyT;          // n1 x (p+2): restriction directions
  const double* ilp_x;       // 1 / lumped degree-p mass per direction (nin)
  const double* ilp_y;
  const double* il1_x;       // 1 / lumped degree-1 mass per direction (n1)
  const double* il1_y;
  const double* V;           // p = 1 generalized eigenvectors, [iy][k], n1 x n1
  const double* F;           // load vector (ndof)
  const double* scale;       // level-0 source weight of the step k - 1 -> k at entry k (k >= 1)
  HmgDev hmg;                // h-multigrid p = 1 solve (solver option coarse = 1)
  LevelDev lev[kMaxLevels];
};

// work item of one workgroup: a chain of `len` steps at time level `level` of instance `inst`
// starting from point k0 (reads V[k0], writes V[k0+1], ... V[k0+len]); in residual mode one
// step whose result minus V[k0+1] goes to point outj of the next level's right-hand side.
struct PhiJob {
  int inst, level, k0, len, outj;
  int flags;  // bit 0: the job's targets hold no network prediction (guess mode 4 acts as mode 2)
};
// guess modes of PhiParams::guess: 0 zero, 1 previous point, 2 current target (level 0) /
// previous point (coarse levels), 4 the better of the current target and the previous point by
// FP64 residual (level 0; the target then holds a prediction)

enum PhiMode { kModeChain = 0, kModeResidual = 1, kModeGiven = 2 };

struct PhiParams {
  const InstDev* inst;     // device array of instances
  const PhiJob* jobs;      // one per workgroup
  double* const* vtab;     // [inst * kMaxLevels + level] level arrays (points x ndof)
  double* const* gtab;     // [inst * kMaxLevels + level] right-hand sides of coarse levels (null at 0)
  const double* bgiven;    // mode kModeGiven: right-hand sides, job j at bgiven + j * ndof
  double* xgiven;          // mode kModeGiven: guesses in / solutions out
  double* nrm2;            // residual mode: ||r||^2 per workgroup
  int* vcount;             // V-cycles per workgroup (accumulated)
  int* vlast;              // mode kModeGiven: V-cycles of this solve per workgroup (may be null)
  unsigned long long* vinst;  // V-cycles per instance (accumulated since create)
  const int* frozen;          // MGRIT: instances already converged (their jobs return at once; null: none)
  int* status;             // error flags (bit 0 non-finite, bit 1 V-cycle cap)
  double* ws;              // per-workgroup global scratch
  int64_t ws_stride;       // doubles per workgroup
  int mode, guess, maxcyc, nu1, nu2;
  int kshift;              // added to every job's first point (one job list serves all steps)
  int solver;              // 0 p-multigrid, 1 Jacobi-preconditioned CG (FP64)
  int coarse;              // p = 1 solve: 0 exact, 1 one h-multigrid W-cycle
  int64_t hmg_off;         // offset (doubles) of the h-multigrid scratch in a workgroup's slice
  double stol;             // spatial tolerance at level 0
  double stolc;            // spatial tolerance at coarse levels
};

// LDS placement of the work vectors (byte offsets, -1 = global scratch)
struct LdsPlan {
  int off_y, off_d, off_s, off_x, off_sbuf, nmax;
  int zidx;       // index (in V-cycle words) of the always-zero word at the end of the y slot
  int ka;         // off-block entries per lane of the prefetched triangular solves (2, 4, 8, 16)
  int off_win;    // y not in LDS: LDS window of the triangular solves (-1: none)
  int zwin;       // index (in V-cycle words) of the window's always-zero word
  int off_stage = -1;  // staging area of the p = 1 transforms, kStageDoubles (-1: none)
  int off_bst = -1;    // y not in LDS: staging area of the band passes (-1: none)
  int bst_bytes = 0;   // its size
};

enum : int { kY = 1, kD = 2, kS = 4, kX = 8 };
// placement flag: the FP32 spatial-solve kernel built for two 512-thread workgroups per CU (at
// most 128 VGPRs per lane); with an LDS plan of at most half the CU's LDS two chains then share a CU
constexpr int kOcc2 = 16;
// placement flag: the spatial-solve kernel built for 1024-thread workgroups (8 lanes per
// triangular-solve row, slot tables in that layout); y must be in LDS
constexpr int kT1024 = 32;
// placement flag: the 512-thread spatial-solve kernel with 8 lanes per triangular-solve row (the
// 1024-thread build's slot tables, 64 row slots); y must be in LDS and every level of the
// group's schedules must hold at most 64 rows
constexpr int kW8 = 64;
// placement flag: the extended 512-thread build (theta < 1, h-multigrid p = 1 solve, CG), set by
// the library itself whenever a handle uses one of those
constexpr int kExt = 128;

// fixed device scratch of the allocation-free spatial-solve entry point: 64 MiB per device
constexpr int64_t kScratchDoubles = (int64_t)1 << 23;
constexpr int kMaxDevices = 64;

}  // namespace pmg
