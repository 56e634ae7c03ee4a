// device_types.hpp -- plain structs shared by the host driver and the HIP kernels.
#pragma once

#include <cstdint>

namespace pmg {

constexpr int kMaxLevels = 12;   // MGRIT time levels per instance
constexpr int kThreads = 256;    // threads per workgroup of the spatial-solve kernel

// level-scheduled blocked triangular solve (see TriSchedule in host_setup.hpp)
struct TriDev {
  int nlev, bs, max_rows, pad;
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

// one MGRIT time level of one instance: A_l = M + kappa dt_l K and its smoother / coarse data
struct LevelDev {
  double dt;
  const double* A64;   // FP64 values of A_l on the pattern of M (rp/ci of the instance)
  const void* Avt;     // A_l values in the V-cycle precision
  TriDev L, U;         // ILUT(A_l) factors
  const double* tl;    // exact p = 1 solve: Thomas multipliers per mode [n1][n1]
  const double* tdinv; //                    inverse pivots per mode [n1][n1]
};

struct InstDev {
  int ndof, n1, ndof1, nlev;
  int nt, pad0;
  const int* rp;       // CSR pattern shared by M and every A_l
  const int* ci;
  const double* M;     // mass matrix values (FP64)
  const int* Rrp;      // restriction (M1^L)^{-1} P^T: ndof1 x ndof
  const int* Rci;
  const void* Rv;      // V-cycle precision
  const int* Qrp;      // prolongation (Mp^L)^{-1} P: ndof x ndof1
  const int* Qci;
  const void* Qv;
  const double* V;     // p = 1 generalized eigenvectors, [iy][k], n1 x n1
  const double* F;     // load vector (ndof)
  const double* scale; // level-0 source scale dt * tfac(t_k) for k = 0..N_t
  LevelDev lev[kMaxLevels];
};

// work item of one workgroup: a chain of `len` steps at time level `level` of instance `inst`
// starting from point k0 (reads V[k0], writes V[k0+1], ... V[k0+len]); in residual mode one
// step whose result minus V[k0+1] goes to point outj of the next level's right-hand side.
struct PhiJob {
  int inst, level, k0, len, outj, pad;
};

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
  int* status;             // error flags (bit 0 non-finite, bit 1 V-cycle cap)
  double* ws;              // per-workgroup global scratch
  int64_t ws_stride;       // doubles per workgroup
  int mode, guess, maxcyc, nu1, nu2, lds_vec_bytes;
  double stol;
};

}  // namespace pmg
