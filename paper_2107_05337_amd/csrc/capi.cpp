// capi.cpp -- the C ABI (include/pmgrit.h): host setup per instance and time level, upload,
// and the MGRIT driver that enqueues the batched spatial-solve launches on one HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pmgrit.h"
#include "device_types.hpp"
#include "host_setup.hpp"
#include "net.hpp"

namespace pmg {
hipError_t phi_prepare(int fp32, int mask, int lds_bytes);
hipError_t phi_launch(int fp32, int mask, int lds_bytes, const PhiParams& P, const LdsPlan& plan, int nblocks,
                      hipStream_t st);
hipError_t fill_launch(double* p, int64_t n, double v, hipStream_t st);
hipError_t copy_launch(double* dst, const double* src, int64_t n, hipStream_t st);
hipError_t correct_launch(double* Vl, const double* Vc, int ndof, int m, int ncoarse, const int* frozen,
                          hipStream_t st);
hipError_t norm_reduce_launch(const double* nrm2, const int* begin, const int* id, double* out, int ninst,
                              hipStream_t st);
hipError_t scratch_setup(int device);
double* scratch_ptr(int device);
}  // namespace pmg

using namespace pmg;

constexpr int kGivenMax = 1024;  // right-hand sides per pmgrit_phi call

static thread_local std::string g_err;

static pmgrit_status fail(pmgrit_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return fail(PMGRIT_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------------------------------
// host data
// ------------------------------------------------------------------------------------------

struct LevelHost {
  double dt = 0;
  Csr A, L, U;  // A on the pattern of M
  TriSchedule SL, SU;
  std::vector<double> tl, tdinv;
  std::vector<double> htl, htd;  // h-multigrid p = 1 solve: Thomas data of the coarsest h-level
};

// h-multigrid of the p = 1 problem: interior 1D factors Mx, Kx, Mx2, My, Ky per h-level (level 0:
// the rediscretised p = 1 matrices; level k: Galerkin products P^T T P with the 1D canonical
// prolongation), and the coarsest level's eigenvectors for its exact solve
struct HmgHost {
  std::vector<int> ne;                  // elements per direction of each h-level
  std::vector<std::vector<Dense>> T;    // [level][5]
  Dense Vc;
  std::vector<double> lam;
};

struct InstHost {
  pmgrit_problem prob{};
  int p = 0, n = 0, domain = 0, N = 0, Nin = 0, ndof = 0, n1 = 0, ndof1 = 0, nlev = 0;
  std::vector<int> Nl;
  Dense Mx, Kx, Mx2, My, Ky, Px, Py, M1x, K1x, M1x2, M1y, K1y;  // 1D factors
  Csr M, K, P, M1, K1;  // host copies (ILUT input, inspection)
  std::vector<double> mlp, ml1, F, u0, scale;
  int tkind = 0;
  CoarseFdm fdm;
  HmgHost hmg;
  std::vector<LevelHost> lev;
};

struct DevBuf {
  void* p = nullptr;
};

struct pmgrit_handle {
  int device = -1;
  int ncu = 256;  // compute units of the device (sweeps wider than this use the wide placement)
  int ninst = 0;
  pmgrit_mgrit_opts mo{};
  pmgrit_solver_opts so{};
  std::vector<InstHost> inst;
  int nlev = 0, Nt = 0, m = 0;
  std::vector<int> Nl;
  double t_setup = 0;
  // device side
  std::vector<void*> allocs;
  InstDev* d_inst = nullptr;
  std::vector<InstDev> h_instdev;
  double** d_vtab = nullptr;
  double** d_gtab = nullptr;
  std::vector<double*> h_vtab, h_gtab;
  int* d_status = nullptr;
  double* d_resnorm = nullptr;
  // MGRIT: per instance, converged (its jobs and corrections skip it) while freeze_on is set
  int* d_frozen = nullptr;
  int* h_frozen = nullptr;  // pinned host copy of the flags
  bool freeze_on = false;
  double* h_pinned = nullptr;  // residual norms read back per MGRIT iteration
  PhiJob* h_given_jobs = nullptr;
  int given_key[3] = {-1, -1, -1};
  int fp32 = 0;
  int ext = 0;  // kExt: the extended kernel build (theta < 1, h-multigrid p = 1 solve or CG)
  struct JobList {
    PhiJob* d = nullptr;
    int n = 0;
    int64_t steps = 0;  // spatial solves the list performs
  };
  // Instances are grouped by the LDS placement they can use; every group has its own launch
  // configuration, job lists and scratch, and launches on its own stream so that groups of
  // different sizes run concurrently within a sweep.
  struct Group {
    std::vector<int> inst;
    int mask = 0, lds_bytes = 0, nmax = 0, n1max = 0, ka = 2, rw = 8, maxrows = 1;
    int ka8 = 2, rw8 = 16;  // the same for the 1024-thread build (8 lanes per row)
    float tuned_ms = 0.f;  // probe time of the chosen placement (autotune)
    LdsPlan plan{-1, -1, -1, -1, 512, 0, 0, 2, -1, 0};
    int winw = 0;  // LDS window words of the triangular solves when y is not in LDS (0: none)
    // placement of the sweeps with more workgroups than the device has CUs (the level-0 sweeps),
    // where two workgroups per CU can pay; mask / lds_bytes / plan serve the narrower ones
    int wmask = 0, wbytes = 0;
    LdsPlan wplan{-1, -1, -1, -1, 512, 0, 0, 2, -1, 0};
    std::vector<JobList> jF, jC, jRES;  // per level: F-relaxation chains, C-steps, C-point residuals
    JobList jCoarsest, jSeq;
    // single-step lists of the learned warm start: level-0 F steps per position s in the
    // interval, and one step per instance (sequential stepping, shifted by k)
    std::vector<JobList> jF1;
    JobList jC1;  // the level-0 C-steps of the learned first iteration (flags: which are predicted)
    bool netfree = false;  // no instance of the group is predicted by the network in MGRIT
    JobList jSeq1;
    int max_jobs = 0;
    double* d_ws = nullptr;
    int64_t ws_stride = 0;
    int64_t hmg_off = 0;  // h-multigrid scratch offset in a slice
    double* d_nrm2 = nullptr;
    int* d_vcount = nullptr;
    int* d_res_begin = nullptr;  // level-0 residual workgroup ranges per group-local instance
    int* d_res_inst = nullptr;   // their global instance ids
    PhiJob* d_given_jobs = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
  };
  std::vector<Group> groups;
  std::vector<int> launch_order;  // groups by decreasing cost: each sweep launches the costliest first
  // >= 0: the MGRIT driver is issuing one group's work on that group's own stream (sweeps, fills and
  // corrections cover only its instances); -1: every group, joined after each sweep
  int only_group = -1;
  bool skip_netfree = false;  // sweeps leave out the groups marked netfree
  std::vector<int> all_inst;  // 0 .. ninst - 1
  std::vector<int> inst_group;
  // learned warm start: the network and, per grid size, the samples of the single-step lists
  std::unique_ptr<NetState> net;
  struct NetGroup {
    int G = 0;
    std::vector<int> inst;
    NetPick* d_seq = nullptr;  // (i, 0) per instance, shifted by k
    std::vector<NetPick*> d_f;  // per s: level-0 F steps (i, j m + s)
    std::vector<int> nf;
    NetPick* d_c = nullptr;  // level-0 C steps (i, j m - 1)
    int nc = 0;
  };
  std::vector<NetGroup> ngroups;
  NetSrc* d_netsrc = nullptr;
  NetSrc* h_netsrc = nullptr;  // pinned staging
  NetSrc* d_src_tmp = nullptr;
  NetPick* d_pick_tmp = nullptr;
  hipEvent_t fork = nullptr;
  // captured MGRIT iteration (mgrit use_graph) for one set of trajectory buffers and stream
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t gstream = nullptr;  // solve stream of graph mode (the caller's may be the null stream)
  hipEvent_t gfork = nullptr, gjoin = nullptr;
  std::vector<void*> graph_key;
  hipStream_t graph_stream = nullptr;
  int64_t graph_phi = 0, graph_launches = 0, graph_wgs = 0;
  int64_t nlaunch_total = 0, nwg_total = 0;  // spatial-solve launches issued or captured
  // live kernel timing
  bool prof = false;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  std::vector<int> ev_group;  // launch group of each recorded event pair (-1: a graph replay)
  std::vector<double> gprof_ms;             // per launch group: kernel ms, launches, workgroups
  std::vector<int64_t> gprof_launches, gprof_wgs;
  unsigned long long* d_vinst = nullptr;    // V-cycles per instance (device counters)
  double prof_ms = 0;
  int64_t vc_base = 0;  // V-cycle counter total at the last profile reset
  int64_t prof_launches = 0, prof_wgs = 0;
};

// ------------------------------------------------------------------------------------------
// setup of one instance
// ------------------------------------------------------------------------------------------

static Csr transpose(const Csr& A) {
  Csr T;
  T.nr = A.nc;
  T.nc = A.nr;
  T.rp.assign(T.nr + 1, 0);
  for (int j : A.ci) T.rp[j + 1]++;
  for (int i = 0; i < T.nr; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  std::vector<int> pos(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < A.nr; ++i)
    for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
      int j = A.ci[t];
      T.ci[pos[j]] = i;
      T.v[pos[j]] = A.v[t];
      pos[j]++;
    }
  return T;
}

// interior rows of the full row sums of Y kron X
static std::vector<double> lumped(const Dense& Y, const Dense& X) {
  std::vector<double> sy(Y.r, 0.0), sx(X.r, 0.0);
  for (int i = 0; i < Y.r; ++i)
    for (int j = 0; j < Y.c; ++j) sy[i] += Y(i, j);
  for (int i = 0; i < X.r; ++i)
    for (int j = 0; j < X.c; ++j) sx[i] += X(i, j);
  std::vector<double> out;
  for (int iy = 1; iy < Y.r - 1; ++iy)
    for (int ix = 1; ix < X.r - 1; ++ix) out.push_back(sy[iy] * sx[ix]);
  return out;
}

static Dense interior(const Dense& A) {
  Dense B(A.r - 2, A.c - 2);
  for (int i = 1; i < A.r - 1; ++i)
    for (int j = 1; j < A.c - 1; ++j) B(i - 1, j - 1) = A(i, j);
  return B;
}

// Cholesky of a dense SPD matrix (lower), in place
static bool chol(Dense& A) {
  const int n = A.r;
  for (int j = 0; j < n; ++j) {
    double s = A(j, j);
    for (int k = 0; k < j; ++k) s -= A(j, k) * A(j, k);
    if (!(s > 0)) return false;
    A(j, j) = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A(i, j);
      for (int k = 0; k < j; ++k) t -= A(i, k) * A(j, k);
      A(i, j) = t / A(j, j);
    }
    for (int k = j + 1; k < n; ++k) A(j, k) = 0.0;
  }
  return true;
}

// generalized symmetric eigenproblem K v = lam M v with V^T M V = I
static bool gen_eig(const Dense& K, const Dense& M, std::vector<double>& lam, Dense& V) {
  const int n = K.r;
  Dense C = M;
  if (!chol(C)) return false;
  // S = C^{-1} K C^{-T}: solve C W = K (columns), then S = C^{-1} W^T
  Dense W(n, n), S(n, n);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double t = K(i, c);
      for (int k = 0; k < i; ++k) t -= C(i, k) * W(k, c);
      W(i, c) = t / C(i, i);
    }
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double t = W(c, i);
      for (int k = 0; k < i; ++k) t -= C(i, k) * S(k, c);
      S(i, c) = t / C(i, i);
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) S(i, j) = S(j, i) = 0.5 * (S(i, j) + S(j, i));
  Dense Z;
  sym_eig(S, lam, Z);
  // V = C^{-T} Z: back substitution with C^T
  V = Dense(n, n);
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double t = Z(i, c);
      for (int k = i + 1; k < n; ++k) t -= C(k, i) * V(k, c);
      V(i, c) = t / C(i, i);
    }
  return true;
}

static pmgrit_status setup_instance(pmgrit_handle* H, InstHost& I, const pmgrit_problem& pr) {
  I.prob = pr;
  I.p = pr.degree_p;
  I.n = pr.n_elems;
  I.domain = pr.domain;
  const int p = I.p, n = I.n, q = p + 1;
  I.N = n + p;
  I.Nin = n + p - 2;
  I.ndof = I.Nin * I.Nin;
  I.n1 = n - 1;
  I.ndof1 = I.n1 * I.n1;
  // weights of the separable parametrisation: square 1; annulus r(s) = 1 + s (first
  // direction), |c'(t)| (second); the stiffness splits into a radial and an angular term
  const bool ann = I.domain == 1;
  const int wr = ann ? 1 : 0, wri = ann ? 2 : 0, wt = ann ? 3 : 0, wti = ann ? 4 : 0;
  I.Mx = weighted_1d(n, p, p, 0, 0, wr, q);
  I.Kx = weighted_1d(n, p, p, 1, 1, wr, q);
  I.Mx2 = ann ? weighted_1d(n, p, p, 0, 0, wri, q) : I.Mx;
  I.My = weighted_1d(n, p, p, 0, 0, wt, q);
  I.Ky = weighted_1d(n, p, p, 1, 1, wti, q);
  I.Px = weighted_1d(n, p, 1, 0, 0, wr, q);
  I.Py = weighted_1d(n, p, 1, 0, 0, wt, q);
  I.M1x = weighted_1d(n, 1, 1, 0, 0, wr, q);
  I.K1x = weighted_1d(n, 1, 1, 1, 1, wr, q);
  I.M1x2 = ann ? weighted_1d(n, 1, 1, 0, 0, wri, q) : I.M1x;
  I.M1y = weighted_1d(n, 1, 1, 0, 0, wt, q);
  I.K1y = weighted_1d(n, 1, 1, 1, 1, wti, q);
  // 2D operators: M = My x Mx, K = My x Kx + Ky x Mx2, P = Py x Px (y slow, x fast)
  I.M = kron_interior(I.N, I.N, I.N, I.N, -p, p, -p, p, {{&I.My, &I.Mx, 1.0}});
  I.K = kron_interior(I.N, I.N, I.N, I.N, -p, p, -p, p, {{&I.My, &I.Kx, 1.0}, {&I.Ky, &I.Mx2, 1.0}});
  I.P = kron_interior(I.N, I.N, n + 1, n + 1, -p, 1, -p, 1, {{&I.Py, &I.Px, 1.0}});
  I.M1 = kron_interior(n + 1, n + 1, n + 1, n + 1, -1, 1, -1, 1, {{&I.M1y, &I.M1x, 1.0}});
  I.K1 = kron_interior(n + 1, n + 1, n + 1, n + 1, -1, 1, -1, 1, {{&I.M1y, &I.K1x, 1.0}, {&I.K1y, &I.M1x2, 1.0}});
  I.mlp = lumped(I.My, I.Mx);
  I.ml1 = lumped(I.M1y, I.M1x);
  I.F.assign(I.ndof, 0.0);
  I.u0.assign(I.ndof, 0.0);
  // exact p = 1 solve: generalized eigenvectors of the second direction
  {
    Dense My1 = interior(I.M1y), Ky1 = interior(I.K1y);
    Dense V;
    if (!gen_eig(Ky1, My1, I.fdm.lam, V)) return PMGRIT_E_FACTOR;
    I.fdm.n1 = I.n1;
    I.fdm.V = V.a;
  }
  // h-multigrid of the p = 1 problem: halve the mesh while the element count is even and above 4
  if (H->so.coarse == 1) {
    HmgHost& hm = I.hmg;
    for (int ne = n;;) {
      hm.ne.push_back(ne);
      if ((int)hm.ne.size() == kHmgMax || ne % 2 != 0 || ne <= 4) break;
      ne /= 2;
    }
    hm.T.resize(hm.ne.size());
    hm.T[0] = {interior(I.M1x), interior(I.K1x), interior(I.M1x2), interior(I.M1y), interior(I.K1y)};
    for (size_t k = 1; k < hm.ne.size(); ++k) {
      const int nf = hm.ne[k - 1] - 1, nc = hm.ne[k] - 1;
      // canonical prolongation: coarse node J (0-based) is fine node 2J + 1; its hat is 1/2, 1, 1/2
      // on fine nodes 2J, 2J + 1, 2J + 2
      Dense P1(nf, nc);
      for (int J = 0; J < nc; ++J) {
        P1(2 * J, J) = 0.5;
        P1(2 * J + 1, J) = 1.0;
        P1(2 * J + 2, J) = 0.5;
      }
      for (const Dense& Tf : hm.T[k - 1]) {
        Dense TP(nf, nc), C(nc, nc);
        for (int i = 0; i < nf; ++i)
          for (int J = 0; J < nc; ++J) {
            double t = 0.0;
            for (int j = std::max(0, 2 * J - 1); j <= std::min(nf - 1, 2 * J + 3); ++j) t += Tf(i, j) * P1(j, J);
            TP(i, J) = t;
          }
        for (int I2 = 0; I2 < nc; ++I2)
          for (int J = 0; J < nc; ++J) {
            double t = 0.0;
            for (int i = 2 * I2; i <= 2 * I2 + 2; ++i) t += P1(i, I2) * TP(i, J);
            C(I2, J) = t;
          }
        hm.T[k].push_back(C);
      }
    }
    const std::vector<Dense>& Tc = hm.T.back();
    if (!gen_eig(Tc[4], Tc[3], hm.lam, hm.Vc)) return PMGRIT_E_FACTOR;
  }
  // time levels (factored by setup_level, in parallel over instances and levels)
  const double dt0 = pr.T / pr.n_steps;
  I.nlev = H->nlev;
  I.lev.resize(I.nlev);
  I.scale.assign(pr.n_steps + 1, dt0);
  return PMGRIT_OK;
}

// One time level of one instance: A_l = M + kappa dt_l K, ILUT(A_l), the blocked triangular
// schedules of its factors and the Thomas data of the exact p = 1 solve.  Runs on a worker
// thread: reports failures through err instead of the thread-local error message.
static pmgrit_status setup_level(const pmgrit_handle* H, InstHost& I, int l, std::string& err) {
  const pmgrit_problem& pr = I.prob;
  const double dt0 = pr.T / pr.n_steps;
  Dense G1 = interior(I.M1x), K1i = interior(I.K1x), H1 = interior(I.M1x2);
  LevelHost& Lv = I.lev[l];
  Lv.dt = dt0 * std::pow((double)H->m, l);
  // theta-scheme (Sec. 2, eq:los): the solves invert A_l = M + theta kappa dt_l K
  const double c = pr.theta * pr.kappa * Lv.dt;
  Lv.A = I.M;
  for (size_t t = 0; t < Lv.A.v.size(); ++t) Lv.A.v[t] = I.M.v[t] + c * I.K.v[t];
  std::vector<int> lc(I.ndof), uc(I.ndof);
  for (int i = 0; i < I.ndof; ++i) {
    int lo = 0, up = 0;
    for (int t = Lv.A.rp[i]; t < Lv.A.rp[i + 1]; ++t) {
      lo += Lv.A.ci[t] < i;
      up += Lv.A.ci[t] > i;
    }
    lc[i] = lo;
    uc[i] = up;
  }
  if (!ilut(Lv.A, H->so.ilut_droptol, lc, uc, Lv.L, Lv.U, err)) return PMGRIT_E_FACTOR;
  int bs = H->so.trsv_block;
  if (bs == 0) {
    // 64 consecutive rows per block, whatever the grid lines: four full wavefronts of the
    // 512-thread build per level (a 65-row line would leave a fifth wavefront nearly empty, and
    // the level waits for it), and lines shorter than 64 rows share blocks, so fewer levels.
    // Instances whose FP64-sized triangular-solve vector cannot be in LDS run in window mode, where
    // each level waits on table loads from HBM: blocks of 128 rows halve the dependent levels.
    // (FP32 V-cycles only: the FP64 window solve keeps 64-row blocks, see kWinDense)
    const bool window = (int64_t)I.ndof * 8 + 16 + 512 + kSbufWords * 8 > (int64_t)kLdsBytes;
    bs = std::min(I.ndof, window ? kWinBlock : kWaveBlock);
  } else if (bs == -1) {
    // one grid line per block, split evenly when a line exceeds the prefetched path's 72 rows
    const int parts = (I.Nin + kDenseMax - 1) / kDenseMax;
    bs = (I.Nin + parts - 1) / parts;
  }
  // at most kRowSlots rows per level, the prefetched path's row slots
  Lv.SL = build_schedule(Lv.L, false, bs, kRowSlots);
  Lv.SU = build_schedule(Lv.U, true, bs, kRowSlots);
  // Thomas data per mode k: T_k = G + c lam_k H with G = M1x + c K1x
  const int n1 = I.n1;
  Lv.tl.assign((size_t)n1 * n1, 0.0);
  Lv.tdinv.assign((size_t)n1 * n1, 0.0);
  for (int k = 0; k < n1; ++k) {
    double dprev = 0.0;
    for (int i = 0; i < n1; ++i) {
      double diag = G1(i, i) + c * K1i(i, i) + c * I.fdm.lam[k] * H1(i, i);
      double li = 0.0;
      if (i > 0) {
        double off = G1(i, i - 1) + c * K1i(i, i - 1) + c * I.fdm.lam[k] * H1(i, i - 1);
        li = off / dprev;
        diag -= li * off;
      }
      if (!(diag > 0)) {
        err = "p=1 tridiagonal not SPD";
        return PMGRIT_E_FACTOR;
      }
      Lv.tl[(size_t)k * n1 + i] = li;
      Lv.tdinv[(size_t)k * n1 + i] = 1.0 / diag;
      dprev = diag;
    }
  }
  if (H->so.coarse == 1) {
    // coarsest h-level: modes of (Mx + c Kx) + c lam_k Mx2 as above
    const std::vector<Dense>& Tc = I.hmg.T.back();
    const int nc = Tc[0].r;
    Lv.htl.assign((size_t)nc * nc, 0.0);
    Lv.htd.assign((size_t)nc * nc, 0.0);
    for (int k = 0; k < nc; ++k) {
      double dprev = 0.0;
      for (int i = 0; i < nc; ++i) {
        const double lk = I.hmg.lam[k];
        double diag = Tc[0](i, i) + c * Tc[1](i, i) + c * lk * Tc[2](i, i);
        double li = 0.0;
        if (i > 0) {
          const double off = Tc[0](i, i - 1) + c * Tc[1](i, i - 1) + c * lk * Tc[2](i, i - 1);
          li = off / dprev;
          diag -= li * off;
        }
        if (!(diag > 0)) {
          err = "coarsest h-multigrid tridiagonal not SPD";
          return PMGRIT_E_FACTOR;
        }
        Lv.htl[(size_t)k * nc + i] = li;
        Lv.htd[(size_t)k * nc + i] = 1.0 / diag;
        dprev = diag;
      }
    }
  }
  return PMGRIT_OK;
}

// run f(t) for t in [0, ntask) on up to 16 host threads; returns the first failure
template <class F>
static pmgrit_status parallel_tasks(int ntask, F f, std::string& err) {
  std::atomic<int> next{0};
  std::mutex mu;
  pmgrit_status first = PMGRIT_OK;
  auto worker = [&]() {
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= ntask) return;
      std::string e;
      const pmgrit_status s = f(t, e);
      if (s != PMGRIT_OK) {
        std::lock_guard<std::mutex> lk(mu);
        if (first == PMGRIT_OK) {
          first = s;
          err = e;
        }
      }
    }
  };
  int nth = (int)std::thread::hardware_concurrency();
  nth = std::max(1, std::min({nth, 16, ntask}));
  std::vector<std::thread> pool;
  for (int i = 1; i < nth; ++i) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  return first;
}

// host version of the exact p = 1 solve (for testing the setup)
static void host_coarse_solve(const InstHost& I, int level, const double* b, double* x) {
  const int n1 = I.n1;
  const LevelHost& L = I.lev[level];
  std::vector<double> c((size_t)n1 * n1);
  for (int k = 0; k < n1; ++k)
    for (int ix = 0; ix < n1; ++ix) {
      double s = 0;
      for (int iy = 0; iy < n1; ++iy) s += I.fdm.V[(size_t)iy * n1 + k] * b[(size_t)iy * n1 + ix];
      c[(size_t)k * n1 + ix] = s;
    }
  for (int k = 0; k < n1; ++k) {
    double* rw = &c[(size_t)k * n1];
    const double* tl = &L.tl[(size_t)k * n1];
    const double* td = &L.tdinv[(size_t)k * n1];
    double yp = rw[0];
    rw[0] = yp * td[0];
    for (int i = 1; i < n1; ++i) {
      double yv = rw[i] - tl[i] * yp;
      rw[i] = yv * td[i];
      yp = yv;
    }
    for (int i = n1 - 2; i >= 0; --i) rw[i] -= tl[i + 1] * rw[i + 1];
  }
  for (int iy = 0; iy < n1; ++iy)
    for (int ix = 0; ix < n1; ++ix) {
      double s = 0;
      for (int k = 0; k < n1; ++k) s += I.fdm.V[(size_t)iy * n1 + k] * c[(size_t)k * n1 + ix];
      x[(size_t)iy * n1 + ix] = s;
    }
}

// ------------------------------------------------------------------------------------------
// device upload
// ------------------------------------------------------------------------------------------

template <typename T>
static pmgrit_status upload(pmgrit_handle* H, const T* src, size_t n, T** dst) {
  *dst = nullptr;
  if (n == 0) n = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) return fail(PMGRIT_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  H->allocs.push_back(p);
  if (src) {
    e = hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(PMGRIT_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  *dst = (T*)p;
  return PMGRIT_OK;
}

template <typename T>
static pmgrit_status upload_vec(pmgrit_handle* H, const std::vector<T>& v, T** dst) {
  return upload(H, v.empty() ? nullptr : v.data(), v.size(), dst);
}

// values in the V-cycle precision
static pmgrit_status upload_vals(pmgrit_handle* H, const std::vector<double>& v, const void** dst) {
  if (H->fp32) {
    std::vector<float> f(v.begin(), v.end());
    float* d = nullptr;
    pmgrit_status s = upload_vec(H, f, &d);
    *dst = d;
    return s;
  }
  double* d = nullptr;
  pmgrit_status s = upload_vec(H, v, &d);
  *dst = d;
  return s;
}

#define TRY(x)                    \
  do {                            \
    pmgrit_status s_ = (x);       \
    if (s_ != PMGRIT_OK) return s_; \
  } while (0)

// winW > 0: window mode, off-block columns become slots of an LDS window of winW grid lines of winN
// rows (line j at slot j mod winW).  Valid when the grid lines each level writes advance
// monotonically (up for L, down for U) and each level's rows and off-block columns span at most
// winW lines: a level then overwrites only the slots of lines no later level reads (a block may
// straddle two lines when a line is split into blocks)
static bool window_fits(const TriSchedule& S, int winW, int winN) {
  int pa = -1, pb = -1, dir = 0;
  for (int l = 0; l < S.nlev; ++l) {
    int a = INT32_MAX, b = -1, lo = INT32_MAX, hi = -1;
    for (int q = S.lev_ptr[l]; q < S.lev_ptr[l + 1]; ++q) {
      const int line = S.row[q] / winN;
      a = std::min(a, line);
      b = std::max(b, line);
      for (int k = S.orp[q]; k < S.orp[q + 1]; ++k) {
        lo = std::min(lo, S.oci[k] / winN);
        hi = std::max(hi, S.oci[k] / winN);
      }
    }
    if (b < 0) continue;
    if (std::max(b, hi) - std::min(a, lo) > winW - 1) return false;
    if (pb >= 0) {
      const int d = (a > pa || b > pb) ? 1 : (a < pa || b < pb) ? -1 : 0;
      if (d != 0) {
        if ((d > 0 && (a < pa || b < pb)) || (d < 0 && (a > pa || b > pb))) return false;
        if (dir != 0 && d != dir) return false;
        dir = d;
      }
    }
    pa = a;
    pb = b;
  }
  return true;
}

static pmgrit_status upload_tri(pmgrit_handle* H, const TriSchedule& S, TriDev& T, int zidx, int RW, int TG, int winW,
                                int winN) {
  T.nlev = S.nlev;
  T.bs = S.bs;
  T.max_rows = S.max_rows;
  // the prefetched register path holds one row per 8 lanes (128 rows per level), up to 64
  // off-block entries per row and dense rows of up to 72 entries starting below word 65536
  int maxo = 0, maxd = 0;
  for (size_t q = 0; q + 1 < S.orp.size(); ++q) maxo = std::max(maxo, S.orp[q + 1] - S.orp[q]);
  for (int c : S.dcnt) maxd = std::max(maxd, c);
  int maxq = 0;  // the dense start column travels in 16 bits of the slot metadata
  for (int c : S.dq0) maxq = std::max(maxq, c);
  const size_t aslots = ((size_t)S.nlev * std::max(1, S.max_rows) + 1) * (size_t)RW;
  T.fast = (zidx >= 0 && S.max_rows <= kRowSlots && maxo <= RW && maxo <= kOffMax &&
            maxd <= (winW > 0 ? kDenseWin : kDenseMax) &&
            maxq < 65536 && S.dval.size() + 1 < (size_t)INT32_MAX && aslots * sizeof(double) < (size_t)kBufBytes &&
            (winW == 0 || window_fits(S, winW, winN)))
               ? 1
               : 0;
  T.winW = T.fast ? winW : 0;
  T.winN = winN;
  auto colmap = [&](int c) { return T.winW ? (c / winN % winW) * winN + c % winN : c; };
  int* p;
  TRY(upload_vec(H, S.lev_ptr, &p));
  T.lev_ptr = p;
  TRY(upload_vec(H, S.row, &p));
  T.row = p;
  TRY(upload_vec(H, S.orp, &p));
  T.orp = p;
  TRY(upload_vec(H, S.oci, &p));
  T.oci = p;
  TRY(upload_vals(H, S.ov, &T.ov));
  TRY(upload_vec(H, S.dq0, &p));
  T.dq0 = p;
  TRY(upload_vec(H, S.dcnt, &p));
  T.dcnt = p;
  // dense values with a reserved zero at index 0 (offsets shifted by one)
  std::vector<double> dval(S.dval.size() + 1, 0.0);
  std::copy(S.dval.begin(), S.dval.end(), dval.begin() + 1);
  std::vector<int64_t> doff(S.doff.size());
  for (size_t q = 0; q < S.doff.size(); ++q) doff[q] = S.doff[q] + 1;
  int64_t* p64;
  TRY(upload_vec(H, doff, &p64));
  T.doff = p64;
  TRY(upload_vals(H, dval, &T.dval));
  if (T.fast) {
    // slot tables: entry 0 reserved (empty slot / zero coefficient whose column is the LDS
    // zero word); level l, row slot r at 1 + l * R + r.  Off-block rows: AS = ka * TG entries in
    // their natural order, zero-padded.  Dense rows: the columns from bq0 rounded down to 16
    // bytes (zeros in front) in natural order, zero-padded to a multiple of TG 16-byte units;
    // bc = values per lane.  The kernel's lane g of TG per row reads 16-byte units g, g + TG, ...
    const int R = std::max(1, S.max_rows), AS = RW, TGh = TG;
    const int V = H->fp32 ? 4 : 2;  // values per 16 bytes
    // records past the last level are empty (the window mode's slab solve reads up to nlev + 2)
    const size_t nslots = (size_t)(S.nlev + 3) * R + 1;
    std::vector<Meta4> meta(nslots, Meta4{-1, 0, 0, 0});
    std::vector<int> acol(aslots, 0);  // columns relative to the zero word zidx (padding: 0)
    std::vector<double> aval(aslots, 0.0);
    std::vector<double> dfast((size_t)TGh * V, 0.0);  // a zero row of one vector per lane at 0
    meta[0] = Meta4{-1, 0, 0, 0};
    for (int l = 0; l < S.nlev; ++l)
      for (int q = S.lev_ptr[l]; q < S.lev_ptr[l + 1]; ++q) {
        const int r = q - S.lev_ptr[l];
        const size_t sl = (size_t)l * R + r;
        const int na = S.orp[q + 1] - S.orp[q];
        const int q0 = S.dq0[q] / V * V, lead = S.dq0[q] - q0, cnt = S.dcnt[q] + lead;
        const int bc = (cnt + TGh * V - 1) / (TGh * V) * V;
        const size_t bo = dfast.size();
        if ((bo + (size_t)TGh * bc) * sizeof(double) >= (size_t)kBufBytes)
          return fail(PMGRIT_E_OOM, "dense table too large");
        dfast.resize(bo + (size_t)TGh * bc, 0.0);
        for (int c = 0; c < S.dcnt[q]; ++c) dfast[bo + lead + c] = S.dval[S.doff[q] + c];
        meta[1 + sl] = Meta4{S.row[q], (int)bo, q0 | (bc << 16), na};
        for (int t = 0; t < na; ++t) {
          aval[(1 + sl) * AS + t] = S.ov[S.orp[q] + t];
          acol[(1 + sl) * AS + t] = colmap(S.oci[S.orp[q] + t]) - zidx;
        }
      }
    // window mode, 512 threads of 4 lanes per row: slab tables when a level's dense rows fit kDch
    // chunks (twice as many in FP64) and the window columns 16 bits
    T.dch = 0;
    T.lsv = 0;
    T.acol16 = nullptr;
    const int vb = H->fp32 ? 4 : 8, dchmax = H->fp32 ? kDch : 2 * kDch;
    if (T.winW > 0 && TGh == 4 && R * TGh == 512 && AS % TGh == 0) {
      size_t maxlev = 0;
      for (int l = 0; l < S.nlev; ++l) {
        size_t sum = 0;
        for (int q = S.lev_ptr[l]; q < S.lev_ptr[l + 1]; ++q) sum += (size_t)TGh * (meta[1 + (size_t)l * R + (q - S.lev_ptr[l])].bqc >> 16);
        maxlev = std::max(maxlev, sum);
      }
      const int dch = (int)((maxlev * vb + kChunkBytes - 1) / kChunkBytes);
      bool c16 = true;
      for (int c : acol) c16 = c16 && c >= -32768 && c <= 32767;
      const int lsv = std::max(1, dch) * (kChunkBytes / vb);
      const size_t slab_vals = (size_t)kSlab0 + (size_t)S.nlev * lsv;
      if (dch >= 1 && dch <= dchmax && c16 && slab_vals * sizeof(double) < (size_t)kBufBytes) {
        std::vector<double> slab(slab_vals, 0.0);
        for (int l = 0; l < S.nlev; ++l) {
          size_t at = (size_t)kSlab0 + (size_t)l * lsv;
          for (int q = S.lev_ptr[l]; q < S.lev_ptr[l + 1]; ++q) {
            Meta4& m = meta[1 + (size_t)l * R + (q - S.lev_ptr[l])];
            const size_t len = (size_t)TGh * (m.bqc >> 16);
            std::copy(dfast.begin() + m.bo, dfast.begin() + m.bo + len, slab.begin() + at);
            m.bo = (int)at;
            at += len;
          }
        }
        dfast.swap(slab);
        // 16-bit columns, lane-major: entry (k * TG + g) * WA + e of a row at g * KA + k * WA + e
        const int KA = AS / TGh, WA = std::min(KA, V);
        std::vector<short> a16(acol.size(), 0);
        for (size_t sl = 0; sl + 1 < acol.size() / AS; ++sl)
          for (int t = 0; t < AS; ++t) {
            const int k = t / WA / TGh, g = t / WA % TGh, e = t % WA;
            a16[(1 + sl) * AS + g * KA + k * WA + e] = (short)acol[(1 + sl) * AS + t];
          }
        short* p16;
        TRY(upload_vec(H, a16, &p16));
        T.acol16 = p16;
        T.dch = dch;
        T.lsv = lsv;
      }
    }
    // FP64 dense rows wider than the register path takes run only on slab tables
    if (!H->fp32 && maxd > kDenseMax && T.dch == 0) T.fast = 0;
    T.R = R;
    T.AS = AS;
    Meta4* m4;
    TRY(upload_vec(H, meta, &m4));
    T.meta = m4;
    TRY(upload_vals(H, dfast, &T.dfast));
    int* pi;
    TRY(upload_vec(H, acol, &pi));
    T.acol = pi;
    TRY(upload_vals(H, aval, &T.aval));
  }
  return PMGRIT_OK;
}

static pmgrit_status upload_jobs(pmgrit_handle* H, pmgrit_handle::Group& G, const std::vector<PhiJob>& jobs,
                                 pmgrit_handle::JobList& out) {
  out.n = (int)jobs.size();
  out.steps = 0;
  for (const PhiJob& j : jobs) out.steps += j.len;
  G.max_jobs = std::max(G.max_jobs, out.n);
  return upload_vec(H, jobs, &out.d);
}

static Dense transpose_dense(const Dense& A) {
  Dense T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

// an n x n table stored by mode (v[k * n + i]) rewritten by node (out[i * n + k])
static std::vector<double> node_major(const std::vector<double>& v) {
  const size_t n = (size_t)std::llround(std::sqrt((double)v.size()));
  std::vector<double> out(v.size());
  for (size_t k = 0; k < n; ++k)
    for (size_t i = 0; i < n; ++i) out[i * n + k] = v[k * n + i];
  return out;
}

// 1 / (full row sums) on the interior rows: the inverse lumped mass of one direction
static std::vector<double> inv_rowsum_interior(const Dense& A) {
  std::vector<double> out;
  for (int i = 1; i < A.r - 1; ++i) {
    double s = 0.0;
    for (int j = 0; j < A.c; ++j) s += A(i, j);
    out.push_back(1.0 / s);
  }
  return out;
}

// band array of the interior block of a full 1D matrix: row o (interior), entry (o, o + lo + d)
static pmgrit_status upload_band(pmgrit_handle* H, const Dense& full, int lo, int w, BandDev& B) {
  const int nr = full.r - 2, nc = full.c - 2;
  std::vector<double> v((size_t)nr * w, 0.0);
  for (int o = 0; o < nr; ++o)
    for (int d = 0; d < w; ++d) {
      const int j = o + lo + d;
      if (j >= 0 && j < nc) v[(size_t)o * w + d] = full(o + 1, j + 1);
    }
  double* f = nullptr;
  TRY(upload_vec(H, v, &f));
  B.f64 = f;
  TRY(upload_vals(H, v, &B.vt));
  B.rows = nr;
  B.w = w;
  B.lo = lo;
  return PMGRIT_OK;
}

// LDS plan for a launch configuration: the largest set of work vectors that fits, in the order
// y, d, s, x.  y is an FP64-sized slot plus a zero word (it also holds the FP64 Kronecker
// temporaries and a p = 1 vector), s holds a V-cycle vector or an FP64 p = 1 vector.
// A placement without y in LDS gets the triangular solves' LDS window (winw words, 0: none)
// when it fits.
static void add_window(LdsPlan& plan, int& off, int mask, int vt, int winw, int dev_lds) {
  if (!(mask & kY) && winw > 0) {
    const int sz = (winw * vt + 15) / 16 * 16;
    if (off + sz <= dev_lds) {
      plan.off_win = off;
      plan.zwin = winw - 1;
      off += sz;
    }
  }
  // staging area of the p = 1 transforms: over the window (never in use at the same time), extended
  // to its size, or after the work vectors when it fits; none otherwise
  const int st = kStageDoubles * 8;
  if (plan.off_win >= 0) {
    const int end = std::max(off, plan.off_win + st);
    if (end <= dev_lds) {
      plan.off_stage = plan.off_win;
      off = end;
    }
  } else if (off + st <= dev_lds) {
    plan.off_stage = off;
    off += st;
  }
  // y in global memory: the rest of the budget stages the band passes (at least kBandStageMin)
  if (!(mask & kY)) {
    const int sz = (dev_lds - off) / 16 * 16;
    if (sz >= kBandStageMin) {
      plan.off_bst = off;
      plan.bst_bytes = sz;
      off += sz;
    }
  }
}

static void lds_plan(int nmax, int n1max, int maxrows, int vt, int ka, int dev_lds, int winw, int& mask, int& bytes,
                     LdsPlan& out) {
  auto al = [](int b) { return (b + 15) / 16 * 16; };
  const int base = 512 + al(std::max(maxrows, kSbufWords) * vt);  // block-sum scratch, sbuf
  const int sz_y = al(nmax * 8 + 16), sz_d = al(nmax * vt), sz_s = al(std::max(nmax * vt, n1max * 8)),
            sz_x = al(nmax * 8);
  const int masks[5] = {15, 7, 3, 1, 0};
  for (int mi = 0; mi < 5; ++mi) {
    const int mk = masks[mi];
    int off = base;
    LdsPlan plan{-1, -1, -1, -1, 512, nmax, nmax * 8 / vt, ka, -1, 0};
    if (mk & kY) { plan.off_y = off; off += sz_y; }
    if (mk & kD) { plan.off_d = off; off += sz_d; }
    if (mk & kS) { plan.off_s = off; off += sz_s; }
    if (mk & kX) { plan.off_x = off; off += sz_x; }
    add_window(plan, off, mk, vt, winw, dev_lds);
    if (off <= dev_lds || mk == 0) {
      mask = mk;
      bytes = off;
      out = plan;
      return;
    }
  }
}

// LDS plan with exactly the vectors of `mask` in LDS (bytes = 0 when it does not fit)
static LdsPlan lds_plan_mask(int nmax, int n1max, int maxrows, int vt, int ka, int dev_lds, int winw, int mask,
                             int& bytes) {
  auto al = [](int b) { return (b + 15) / 16 * 16; };
  int off = 512 + al(std::max(maxrows, kSbufWords) * vt);
  LdsPlan plan{-1, -1, -1, -1, 512, nmax, nmax * 8 / vt, ka, -1, 0};
  if (mask & kY) { plan.off_y = off; off += al(nmax * 8 + 16); }
  if (mask & kD) { plan.off_d = off; off += al(nmax * vt); }
  if (mask & kS) { plan.off_s = off; off += al(std::max(nmax * vt, n1max * 8)); }
  if (mask & kX) { plan.off_x = off; off += al(nmax * 8); }
  // the two-workgroups-per-CU build must keep its plan within half the CU's LDS
  add_window(plan, off, mask, vt, winw, (mask & kOcc2) ? dev_lds / 2 : dev_lds);
  bytes = off <= dev_lds ? off : 0;
  return plan;
}

static int inst_maxrows(const InstHost& I) {
  int r = 1;
  for (const LevelHost& Lh : I.lev) r = std::max(r, std::max(Lh.SL.max_rows, Lh.SU.max_rows));
  return r;
}

static int inst_max_offblock(const InstHost& I) {
  int maxo = 1;
  for (const LevelHost& Lh : I.lev)
    for (const TriSchedule* S : {&Lh.SL, &Lh.SU})
      for (size_t q = 0; q + 1 < S->orp.size(); ++q) maxo = std::max(maxo, S->orp[q + 1] - S->orp[q]);
  return maxo;
}

// sample sources and single-step job / sample lists of the learned warm start
static pmgrit_status learned_setup(pmgrit_handle* H) {
  HIPCHK(hipHostMalloc((void**)&H->h_netsrc, sizeof(NetSrc) * H->ninst, 0));
  for (int i = 0; i < H->ninst; ++i) {
    const InstHost& I = H->inst[i];
    const InstDev& D = H->h_instdev[i];
    NetSrc& S = H->h_netsrc[i];
    std::memset(&S, 0, sizeof(S));
    S.F = D.F;
    S.ilx = D.ilp_x;
    S.ily = D.ilp_y;
    S.scale = D.scale;
    S.My = D.My.f64;
    S.Ky = D.Ky.f64;
    S.Kx = D.Kx.f64;
    S.Mx2 = D.Mx2.f64;
    S.dt = I.lev[0].dt;
    S.kdt = I.prob.kappa * S.dt;
    S.lnc = std::log(S.kdt * (double)I.prob.n_elems * (double)I.prob.n_elems) / 4.0;
    S.nin = I.Nin;
    S.G = I.Nin + 2;
    S.p = I.p;
    S.bw = 2 * I.p + 1;
  }
  TRY(upload<NetSrc>(H, nullptr, (size_t)H->ninst, &H->d_netsrc));
  TRY(upload<NetSrc>(H, nullptr, 1, &H->d_src_tmp));
  TRY(upload<NetPick>(H, nullptr, kGivenMax, &H->d_pick_tmp));
  if (H->so.guess != 3) return PMGRIT_OK;
  const int m = H->m, N0 = H->Nl[0];
  // MGRIT predicts only instances of at most kNetMaxElems elements per direction: at 128 and 256 the
  // previous point already needs as few V-cycles per solve as the network's guess (2.0 against 2.0
  // measured), and the inference's cost grows with the grid.  The others run their level-0 F-chains
  // whole and take their targets (the previous iterate) as the guess
  auto net_on = [&](int i) { return H->inst[i].prob.n_elems <= kNetMaxElems; };
  auto fsteps = [&](int i, int s, auto emit) {
    for (int j = 0; j * m + s + 1 <= N0 && s + 1 < m; ++j) emit(i, j * m + s);
  };
  auto csteps = [&](int i, auto emit) {
    for (int j = 1; j * m <= N0; ++j) emit(i, j * m - 1);
  };
  for (pmgrit_handle::Group& G : H->groups) {
    G.netfree = std::none_of(G.inst.begin(), G.inst.end(), net_on);
    G.jF1.resize(std::max(m - 1, 1));
    for (int s = 0; s + 1 < m; ++s) {
      std::vector<PhiJob> J;
      for (int i : G.inst) {
        if (net_on(i)) {
          fsteps(i, s, [&](int ii, int k) { J.push_back({ii, 0, k, 1, 0, 0}); });
        } else if (s == 0) {
          for (int j = 0; j * m < N0; ++j) {
            const int len = std::min(m - 1, N0 - j * m);
            if (len > 0) J.push_back({i, 0, j * m, len, 0, 1});
          }
        }
      }
      TRY(upload_jobs(H, G, J, G.jF1[s]));
    }
    std::vector<PhiJob> C1;
    for (int i : G.inst)
      for (int j = 1; j * m <= N0; ++j) C1.push_back({i, 0, j * m - 1, 1, 0, net_on(i) ? 0 : 1});
    TRY(upload_jobs(H, G, C1, G.jC1));
    std::vector<PhiJob> S1;
    for (int i : G.inst) S1.push_back({i, 0, 0, 1, 0, 0});
    TRY(upload_jobs(H, G, S1, G.jSeq1));
  }
  // network batches: instances of one grid size
  for (int i = 0; i < H->ninst; ++i) {
    const int Gi = H->inst[i].Nin + 2;
    auto it = std::find_if(H->ngroups.begin(), H->ngroups.end(),
                           [Gi](const pmgrit_handle::NetGroup& N) { return N.G == Gi; });
    if (it == H->ngroups.end()) {
      H->ngroups.emplace_back();
      H->ngroups.back().G = Gi;
      it = H->ngroups.end() - 1;
    }
    it->inst.push_back(i);
  }
  for (pmgrit_handle::NetGroup& N : H->ngroups) {
    std::vector<NetPick> seq, c;
    for (int i : N.inst) {
      seq.push_back({i, 0});
      if (net_on(i)) csteps(i, [&](int ii, int k) { c.push_back({ii, k}); });
    }
    TRY(upload_vec(H, seq, &N.d_seq));
    TRY(upload_vec(H, c, &N.d_c));
    N.nc = (int)c.size();
    N.d_f.assign(std::max(m - 1, 1), nullptr);
    N.nf.assign(std::max(m - 1, 1), 0);
    for (int s = 0; s + 1 < m; ++s) {
      std::vector<NetPick> f;
      for (int i : N.inst)
        if (net_on(i)) fsteps(i, s, [&](int ii, int k) { f.push_back({ii, k}); });
      TRY(upload_vec(H, f, &N.d_f[s]));
      N.nf[s] = (int)f.size();
    }
  }
  return PMGRIT_OK;
}

static pmgrit_status device_setup(pmgrit_handle* H) {
  HIPCHK(hipSetDevice(H->device));
  // address of this device's fixed scratch (the allocation-free entry point), resolved once per device
  HIPCHK(scratch_setup(H->device));
  H->fp32 = H->so.precision == 1;
  H->ext = 0;
  if (H->so.coarse == 1 || H->so.solver == 1) H->ext = kExt;
  for (const InstHost& I : H->inst)
    if (I.prob.theta != 1.0) H->ext = kExt;
  if (H->ext && (H->so.lds_mask & (kOcc2 | kT1024 | kW8)))
    return fail(PMGRIT_E_ARG, "theta < 1, the h-multigrid p = 1 solve and CG run on the 512-thread build only");
  const int vt = H->fp32 ? 4 : 8;
  int dev_lds = 0;
  HIPCHK(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, H->device));
  HIPCHK(hipDeviceGetAttribute(&H->ncu, hipDeviceAttributeMultiprocessorCount, H->device));
  // group the instances by the LDS placement each would get on its own
  H->inst_group.assign(H->ninst, -1);
  {
    std::vector<int> mk(H->ninst);
    for (int i = 0; i < H->ninst; ++i) {
      const InstHost& I = H->inst[i];
      int bytes;
      LdsPlan pl;
      lds_plan(I.ndof, I.ndof1, inst_maxrows(I), vt, 16, dev_lds, (I.p + 3) * I.Nin + 1, mk[i], bytes, pl);
    }
    for (int want : {15, 7, 3, 1, 0}) {
      pmgrit_handle::Group G;
      for (int i = 0; i < H->ninst; ++i)
        if (mk[i] == want) G.inst.push_back(i);
      if (G.inst.empty()) continue;
      // costliest instances first: workgroups are dispatched in job order, so when a sweep has
      // more jobs than CUs the cheaper chains fill the later rounds
      auto cost = [&](int i) { return (double)H->inst[i].ndof * (2 * H->inst[i].p + 1); };
      std::stable_sort(G.inst.begin(), G.inst.end(), [&](int a, int b) { return cost(a) > cost(b); });
      for (int i : G.inst) {
        const InstHost& I = H->inst[i];
        G.nmax = std::max(G.nmax, I.ndof);
        G.n1max = std::max(G.n1max, I.ndof1);
        G.maxrows = std::max(G.maxrows, inst_maxrows(I));
        // off-block entries per lane of the prefetched triangular solves: the widest ILUT row
        // of the group's instances over the 4 (or 8) lanes per row, rounded up
        const int maxo = inst_max_offblock(I);
        // ka in {2, 4, 8, 12, 16}: 16-byte units of 4 entries per lane beyond 2
        auto ka_for = [](int need) { return need <= 2 ? 2 : std::min(16, (need + 3) / 4 * 4); };
        G.ka = std::max(G.ka, ka_for((maxo + 3) / 4));
        G.ka8 = std::max(G.ka8, ka_for((maxo + 7) / 8));
        // LDS window of the triangular solves when y is not in LDS: p + 3 grid lines and a zero word
        G.winw = std::max(G.winw, (I.p + 3) * I.Nin + 1);
      }
      G.rw = G.ka * 4;
      G.rw8 = G.ka8 * 8;
      lds_plan(G.nmax, G.n1max, G.maxrows, vt, G.ka, dev_lds, G.winw, G.mask, G.lds_bytes, G.plan);
      if (H->so.lds_mask) {  // placement chosen by the caller
        int bytes = 0;
        const LdsPlan plan = lds_plan_mask(G.nmax, G.n1max, G.maxrows, vt,
                                           (H->so.lds_mask & (kT1024 | kW8)) ? G.ka8 : G.ka, dev_lds, G.winw,
                                           H->so.lds_mask, bytes);
        if (bytes == 0) return fail(PMGRIT_E_ARG, "lds_mask does not fit a launch group's LDS");
        if ((H->so.lds_mask & kW8) && G.maxrows > kRowSlots / 2)
          return fail(PMGRIT_E_ARG, "lds_mask 64 needs at most 64 rows per triangular-solve level");
        G.mask = H->so.lds_mask;
        G.lds_bytes = bytes;
        G.plan = plan;
      }
      G.mask |= H->ext;
      G.wmask = G.mask;
      G.wbytes = G.lds_bytes;
      G.wplan = G.plan;
      for (int i : G.inst) H->inst_group[i] = (int)H->groups.size();
      H->groups.push_back(std::move(G));
    }
  }
  {
    // the launch groups' cost, n_dof (2p + 1) summed over their instances (the job order's measure)
    std::vector<double> cost(H->groups.size(), 0.0);
    for (size_t g = 0; g < H->groups.size(); ++g)
      for (int i : H->groups[g].inst) cost[g] += (double)H->inst[i].ndof * (2 * H->inst[i].p + 1);
    H->launch_order.resize(H->groups.size());
    for (size_t g = 0; g < H->groups.size(); ++g) H->launch_order[g] = (int)g;
    std::stable_sort(H->launch_order.begin(), H->launch_order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  }
  H->h_instdev.resize(H->ninst);
  for (int i = 0; i < H->ninst; ++i) {
    InstHost& I = H->inst[i];
    InstDev& D = H->h_instdev[i];
    const pmgrit_handle::Group& G = H->groups[H->inst_group[i]];
    std::memset(&D, 0, sizeof(D));
    D.ndof = I.ndof;
    D.n1 = I.n1;
    D.ndof1 = I.ndof1;
    D.nlev = I.nlev;
    D.nt = I.prob.n_steps;
    D.nin = I.Nin;
    D.p = I.p;
    double* d;
    const int p = I.p;
    TRY(upload_band(H, I.Mx, -p, 2 * p + 1, D.Mx));
    TRY(upload_band(H, I.Mx2, -p, 2 * p + 1, D.Mx2));
    TRY(upload_band(H, I.My, -p, 2 * p + 1, D.My));
    TRY(upload_band(H, I.Ky, -p, 2 * p + 1, D.Ky));
    TRY(upload_band(H, I.Kx, -p, 2 * p + 1, D.Kx));
    TRY(upload_band(H, I.Px, -p, p + 2, D.Px));
    TRY(upload_band(H, I.Py, -p, p + 2, D.Py));
    TRY(upload_band(H, transpose_dense(I.Px), -1, p + 2, D.PxT));
    TRY(upload_band(H, transpose_dense(I.Py), -1, p + 2, D.PyT));
    TRY(upload_vec(H, inv_rowsum_interior(I.Mx), &d));
    D.ilp_x = d;
    TRY(upload_vec(H, inv_rowsum_interior(I.My), &d));
    D.ilp_y = d;
    TRY(upload_vec(H, inv_rowsum_interior(I.M1x), &d));
    D.il1_x = d;
    TRY(upload_vec(H, inv_rowsum_interior(I.M1y), &d));
    D.il1_y = d;
    TRY(upload_vec(H, I.fdm.V, &d));
    D.V = d;
    TRY(upload_vec(H, I.F, &d));
    D.F = d;
    TRY(upload_vec(H, I.scale, &d));
    D.scale = d;
    if (H->so.coarse == 1) {
      const HmgHost& hm = I.hmg;
      HmgDev& hd = D.hmg;
      hd.nh = (int)hm.ne.size();
      int64_t words = (int64_t)(hm.ne[0] - 1) * (hm.ne[0] - 1);  // residual temporary
      for (int k = 0; k < hd.nh; ++k) {
        const int n1k = hm.ne[k] - 1;
        hd.n1[k] = n1k;
        if (k > 0) {
          hd.off[k] = words;
          words += 2 * (int64_t)n1k * n1k;
        }
        // [5][n1][3] tridiagonal rows; entries outside the matrix are zero
        std::vector<double> band((size_t)15 * n1k, 0.0);
        for (int mtx = 0; mtx < 5; ++mtx)
          for (int i = 0; i < n1k; ++i)
            for (int dd = -1; dd <= 1; ++dd)
              if (i + dd >= 0 && i + dd < n1k) band[(size_t)3 * (mtx * n1k + i) + dd + 1] = hm.T[k][mtx](i, i + dd);
        TRY(upload_vec(H, band, &d));
        hd.band[k] = d;
      }
      hd.words = words;
      TRY(upload_vec(H, hm.Vc.a, &d));
      hd.Vc = d;
    }
    for (int l = 0; l < I.nlev; ++l) {
      LevelHost& Lh = I.lev[l];
      LevelDev& Ld = D.lev[l];
      Ld.dt = Lh.dt;
      Ld.c = I.prob.theta * I.prob.kappa * Lh.dt;
      Ld.cb = (1.0 - I.prob.theta) * I.prob.kappa * Lh.dt;
      Dense X1 = I.Mx;
      for (size_t t = 0; t < X1.a.size(); ++t) X1.a[t] = I.Mx.a[t] + Ld.c * I.Kx.a[t];
      TRY(upload_band(H, X1, -p, 2 * p + 1, Ld.X1));
      // explicit part B_l = M - (1 - theta) kappa dt_l K = My (x) XB - cb Ky (x) Mx2 (theta < 1)
      if (Ld.cb != 0.0) {
        Dense XB = I.Mx;
        for (size_t t = 0; t < XB.a.size(); ++t) XB.a[t] = I.Mx.a[t] - Ld.cb * I.Kx.a[t];
        TRY(upload_band(H, XB, -p, 2 * p + 1, Ld.XB));
      }
      // the prefetched path reads y from LDS: the y slot, or the window of the last p + 3 grid
      // lines when y is in global memory (the 1024-thread build needs the y slot)
      const bool yl = G.mask & kY, win = !yl && G.plan.off_win >= 0;
      const int zidx = yl ? G.plan.zidx : win ? G.plan.zwin : -1;
      const int wl = win ? I.p + 3 : 0;
      TRY(upload_tri(H, Lh.SL, Ld.L, zidx, G.rw, 4, wl, I.Nin));
      TRY(upload_tri(H, Lh.SU, Ld.U, zidx, G.rw, 4, wl, I.Nin));
      TRY(upload_tri(H, Lh.SL, Ld.L8, yl ? zidx : -1, G.rw8, 8, 0, I.Nin));
      TRY(upload_tri(H, Lh.SU, Ld.U8, yl ? zidx : -1, G.rw8, 8, 0, I.Nin));
      // the Thomas data node-major on the device (one thread per mode reads consecutive words)
      TRY(upload_vec(H, node_major(Lh.tl), &d));
      Ld.tl = d;
      TRY(upload_vec(H, node_major(Lh.tdinv), &d));
      Ld.tdinv = d;
      if (H->so.coarse == 1) {
        TRY(upload_vec(H, node_major(Lh.htl), &d));
        Ld.htl = d;
        TRY(upload_vec(H, node_major(Lh.htd), &d));
        Ld.htd = d;
      }
      if (H->so.solver == 1) {  // diag(A_l) for the Jacobi-preconditioned CG
        std::vector<double> dg(I.ndof, 0.0);
        for (int i = 0; i < I.ndof; ++i)
          for (int t = Lh.A.rp[i]; t < Lh.A.rp[i + 1]; ++t)
            if (Lh.A.ci[t] == i) dg[i] = Lh.A.v[t];
        TRY(upload_vec(H, dg, &d));
        Ld.dgA = d;
      }
    }
  }
  TRY(upload_vec(H, H->h_instdev, &H->d_inst));
  // level arrays: level 0 is the caller's trajectory (table filled per call); coarse levels
  // hold the correction v and the injected right-hand side g
  H->h_vtab.assign((size_t)H->ninst * kMaxLevels, nullptr);
  H->h_gtab.assign((size_t)H->ninst * kMaxLevels, nullptr);
  for (int i = 0; i < H->ninst; ++i)
    for (int l = 1; l < H->nlev; ++l) {
      double* v;
      double* g;
      size_t sz = (size_t)(H->Nl[l] + 1) * H->inst[i].ndof;
      TRY(upload<double>(H, nullptr, sz, &v));
      TRY(upload<double>(H, nullptr, sz, &g));
      HIPCHK(hipMemset(v, 0, sz * sizeof(double)));
      HIPCHK(hipMemset(g, 0, sz * sizeof(double)));
      H->h_vtab[(size_t)i * kMaxLevels + l] = v;
      H->h_gtab[(size_t)i * kMaxLevels + l] = g;
    }
  TRY(upload_vec(H, H->h_vtab, &H->d_vtab));
  TRY(upload_vec(H, H->h_gtab, &H->d_gtab));
  // job lists per group
  const int m = H->m;
  for (pmgrit_handle::Group& G : H->groups) {
    G.jF.resize(H->nlev);
    G.jC.resize(H->nlev);
    G.jRES.resize(H->nlev);
    std::vector<int> res_begin(1, 0);
    for (int l = 0; l + 1 < H->nlev; ++l) {
      // C-relaxation reads the F-points of the preceding F-relaxation, so it is a launch of its
      // own: a fused C-and-F chain would race with the chain of the previous interval, which
      // rewrites the F-point the C-step reads
      std::vector<PhiJob> F, C, RES;
      const int Nl = H->Nl[l];
      for (int i : G.inst) {
        for (int j = 0; j * m < Nl; ++j) {
          int len = std::min(m - 1, Nl - j * m);
          if (len > 0) F.push_back({i, l, j * m, len, 0, 0});
        }
        for (int j = 1; j * m <= Nl; ++j) {
          C.push_back({i, l, j * m - 1, 1, 0, 0});
          RES.push_back({i, l, j * m - 1, 1, j, 0});
        }
        if (l == 0) res_begin.push_back((int)RES.size());
      }
      TRY(upload_jobs(H, G, F, G.jF[l]));
      TRY(upload_jobs(H, G, C, G.jC[l]));
      TRY(upload_jobs(H, G, RES, G.jRES[l]));
    }
    std::vector<PhiJob> C, S;
    for (int i : G.inst) {
      C.push_back({i, H->nlev - 1, 0, H->Nl[H->nlev - 1], 0, 0});
      S.push_back({i, 0, 0, H->Nt, 0, 0});
    }
    TRY(upload_jobs(H, G, C, G.jCoarsest));
    TRY(upload_jobs(H, G, S, G.jSeq));
    if (res_begin.size() != G.inst.size() + 1) res_begin.assign(G.inst.size() + 1, 0);
    TRY(upload_vec(H, res_begin, &G.d_res_begin));
    TRY(upload_vec(H, G.inst, &G.d_res_inst));
    // scratch: one slice per workgroup slot; at least kGivenMax slots for pmgrit_phi
    G.max_jobs = std::max(G.max_jobs, kGivenMax);
    // slice: six vectors of nmax doubles, 32 spare, then the h-multigrid scratch (coarse = 1)
    int64_t hw = 0;
    for (int i : G.inst) hw = std::max(hw, (int64_t)H->h_instdev[i].hmg.words);
    G.hmg_off = 6 * (int64_t)G.nmax + 32;
    G.ws_stride = (G.hmg_off + hw + 31) / 32 * 32;
    TRY(upload<double>(H, nullptr, (size_t)G.ws_stride * G.max_jobs, &G.d_ws));
    TRY(upload<double>(H, nullptr, (size_t)G.max_jobs, &G.d_nrm2));
    TRY(upload<int>(H, nullptr, (size_t)G.max_jobs, &G.d_vcount));
    HIPCHK(hipMemset(G.d_vcount, 0, sizeof(int) * G.max_jobs));
    TRY(upload<PhiJob>(H, nullptr, kGivenMax, &G.d_given_jobs));
    HIPCHK(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&G.done, hipEventDisableTiming));
    HIPCHK(phi_prepare(H->fp32, G.mask, G.lds_bytes));
    HIPCHK(phi_prepare(H->fp32, G.wmask, G.wbytes));
  }
  TRY(learned_setup(H));
  HIPCHK(hipEventCreateWithFlags(&H->fork, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&H->gstream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&H->gfork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&H->gjoin, hipEventDisableTiming));
  TRY(upload<int>(H, nullptr, 4, &H->d_status));
  TRY(upload<double>(H, nullptr, (size_t)H->ninst, &H->d_resnorm));
  TRY(upload<int>(H, nullptr, (size_t)H->ninst, &H->d_frozen));
  HIPCHK(hipMemset(H->d_status, 0, sizeof(int) * 4));
  HIPCHK(hipHostMalloc((void**)&H->h_pinned, sizeof(double) * (H->ninst + 8), 0));
  HIPCHK(hipHostMalloc((void**)&H->h_frozen, sizeof(int) * (H->ninst + 8), 0));
  HIPCHK(hipHostMalloc((void**)&H->h_given_jobs, sizeof(PhiJob) * kGivenMax, 0));
  H->ev.resize(2048);
  for (auto& e : H->ev) HIPCHK(hipEventCreate(&e));
  H->ev_group.assign(H->ev.size() / 2, -1);
  H->gprof_ms.assign(H->groups.size(), 0.0);
  H->gprof_launches.assign(H->groups.size(), 0);
  H->gprof_wgs.assign(H->groups.size(), 0);
  TRY(upload<unsigned long long>(H, nullptr, (size_t)H->ninst, &H->d_vinst));
  HIPCHK(hipMemset(H->d_vinst, 0, sizeof(unsigned long long) * H->ninst));
  HIPCHK(hipDeviceSynchronize());
  return PMGRIT_OK;
}

// ------------------------------------------------------------------------------------------
// driver
// ------------------------------------------------------------------------------------------

static PhiParams base_params(pmgrit_handle* H, const pmgrit_handle::Group& G, int mode, const PhiJob* jobs) {
  PhiParams P;
  std::memset(&P, 0, sizeof(P));
  P.inst = H->d_inst;
  P.jobs = jobs;
  P.vtab = H->d_vtab;
  P.gtab = H->d_gtab;
  P.nrm2 = G.d_nrm2;
  P.vcount = G.d_vcount;
  P.vinst = H->d_vinst;
  P.status = H->d_status;
  P.ws = G.d_ws;
  P.ws_stride = G.ws_stride;
  P.mode = mode;
  P.guess = H->so.guess == 3 ? 2 : H->so.guess;
  P.maxcyc = H->so.max_vcycles;
  P.nu1 = H->so.nu1;
  P.nu2 = H->so.nu2;
  P.stol = H->so.spatial_tol;
  P.stolc = H->so.coarse_tol > 0 ? H->so.coarse_tol : H->so.spatial_tol;
  P.solver = H->so.solver;
  P.coarse = H->so.coarse;
  P.hmg_off = G.hmg_off;
  return P;
}

// accumulate the elapsed times of the recorded event pairs (their streams must be complete)
static hipError_t harvest(pmgrit_handle* H) {
  for (int k = 0; k < H->ev_used; ++k) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, H->ev[2 * k], H->ev[2 * k + 1]);
    if (e != hipSuccess) return e;
    H->prof_ms += ms;
    const int g = H->ev_group[k];
    if (g >= 0) H->gprof_ms[g] += ms;
  }
  H->ev_used = 0;
  return hipSuccess;
}

static hipError_t phi_timed(pmgrit_handle* H, const pmgrit_handle::Group& G, const PhiParams& P, int nblocks,
                            hipStream_t st) {
  H->nlaunch_total++;
  H->nwg_total += nblocks;
  const bool wide = nblocks > H->ncu;
  const int mask = wide ? G.wmask : G.mask, bytes = wide ? G.wbytes : G.lds_bytes;
  const LdsPlan& plan = wide ? G.wplan : G.plan;
  if (!H->prof) return phi_launch(H->fp32, mask, bytes, P, plan, nblocks, st);
  hipError_t e;
  if (H->ev_used * 2 + 2 > (int)H->ev.size()) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    if ((e = harvest(H)) != hipSuccess) return e;
  }
  const int k = H->ev_used++;
  const int gi = (int)(&G - H->groups.data());
  H->ev_group[k] = gi;
  if ((e = hipEventRecord(H->ev[2 * k], st)) != hipSuccess) return e;
  if ((e = phi_launch(H->fp32, mask, bytes, P, plan, nblocks, st)) != hipSuccess) return e;
  H->prof_launches++;
  H->prof_wgs += nblocks;
  H->gprof_launches[gi]++;
  H->gprof_wgs[gi] += nblocks;
  return hipEventRecord(H->ev[2 * k + 1], st);
}

// whether the driver is issuing work for launch group gi
static bool drives(const pmgrit_handle* H, int gi) {
  if (H->only_group >= 0) return gi == H->only_group;
  return !(H->skip_netfree && H->groups[gi].netfree);
}

// one sweep: the given job list of every group, groups concurrently on their own streams
// (fork and join through events on the caller's stream)
template <class Pick>
static hipError_t sweep(pmgrit_handle* H, Pick pick, int mode, hipStream_t st, int guess = -1, int kshift = 0) {
  hipError_t e;
  if (H->only_group >= 0) {
    pmgrit_handle::Group& G = H->groups[H->only_group];
    const pmgrit_handle::JobList& J = pick(G);
    if (J.n == 0) return hipSuccess;
    PhiParams P = base_params(H, G, mode, J.d);
    if (H->freeze_on) P.frozen = H->d_frozen;
    if (guess >= 0) P.guess = guess;
    P.kshift = kshift;
    return phi_timed(H, G, P, J.n, st);
  }
  int active = 0;
  for (int gi = 0; gi < (int)H->groups.size(); ++gi) active += drives(H, gi) && pick(H->groups[gi]).n > 0;
  if (active == 0) return hipSuccess;
  const bool fork = active > 1;
  if (fork && (e = hipEventRecord(H->fork, st)) != hipSuccess) return e;
  for (int gi : H->launch_order) {
    pmgrit_handle::Group& G = H->groups[gi];
    const pmgrit_handle::JobList& J = pick(G);
    if (J.n == 0 || !drives(H, gi)) continue;
    hipStream_t gs = fork ? G.stream : st;
    if (fork && (e = hipStreamWaitEvent(gs, H->fork, 0)) != hipSuccess) return e;
    PhiParams P = base_params(H, G, mode, J.d);
    if (H->freeze_on) P.frozen = H->d_frozen;
    if (guess >= 0) P.guess = guess;
    P.kshift = kshift;
    if ((e = phi_timed(H, G, P, J.n, gs)) != hipSuccess) return e;
    if (fork && (e = hipEventRecord(G.done, gs)) != hipSuccess) return e;
  }
  if (fork)
    for (int gi = 0; gi < (int)H->groups.size(); ++gi)
      if (drives(H, gi) && pick(H->groups[gi]).n > 0 &&
          (e = hipStreamWaitEvent(st, H->groups[gi].done, 0)) != hipSuccess)
        return e;
  return hipSuccess;
}

static int64_t sweep_steps(pmgrit_handle* H, int kind, int l) {
  int64_t s = 0;
  for (int gi = 0; gi < (int)H->groups.size(); ++gi) {
    if (!drives(H, gi)) continue;
    pmgrit_handle::Group& G = H->groups[gi];
    s += kind == 0 ? G.jF[l].steps : kind == 1 ? G.jC[l].steps : kind == 2 ? G.jRES[l].steps
                                                                          : kind == 3 ? G.jCoarsest.steps : G.jSeq.steps;
  }
  return s;
}

// the instances the driver is issuing fills and corrections for (all, or those of the group of
// only_group; skip_netfree is set only around the first relaxation, which has neither)
static const std::vector<int>& driven(pmgrit_handle* H) {
  return H->only_group >= 0 ? H->groups[H->only_group].inst : H->all_inst;
}

// learned guesses written into the targets of a single-step list: which 0 sequential (shifted by
// kbase), 1 level-0 F steps at position s, 2 level-0 C steps
static hipError_t net_predict(pmgrit_handle* H, int which, int s, int kbase, hipStream_t st) {
  for (pmgrit_handle::NetGroup& N : H->ngroups) {
    const NetPick* pk = which == 0 ? N.d_seq : which == 1 ? N.d_f[s] : N.d_c;
    const int nb = which == 0 ? (int)N.inst.size() : which == 1 ? N.nf[s] : N.nc;
    if (nb == 0) continue;
    hipError_t e = H->net->predict(H->d_netsrc, pk, kbase, nb, N.G, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t level_solve(pmgrit_handle* H, int l, int kind, hipStream_t st, int64_t& phi);

// One MGRIT cycle at level l >= 1 on A^{(l)} v = g from the current v (Sec. 3, the MGRIT
// recursion): FCF-relaxation, the C-point residual injected into level l + 1, the level-(l + 1)
// correction from zero by level_solve of the same cycle kind, the C-point update and the
// interpolating F-relaxation.
static hipError_t mgrit_cycle(pmgrit_handle* H, int l, int kind, hipStream_t st, int64_t& phi) {
  hipError_t e;
  auto fl = [l](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jF[l]; };
  // FCF-relaxation, then the C-point residuals injected into the next level
  if ((e = sweep(H, fl, kModeChain, st)) != hipSuccess) return e;
  if ((e = sweep(H, [l](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jC[l]; }, kModeChain, st)) !=
      hipSuccess)
    return e;
  if ((e = sweep(H, fl, kModeChain, st)) != hipSuccess) return e;
  if ((e = sweep(H, [l](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jRES[l]; }, kModeResidual,
                 st)) != hipSuccess)
    return e;
  // F, C, F, residual (the interpolating F-relaxation is counted where it is launched)
  phi += 2 * sweep_steps(H, 0, l) + sweep_steps(H, 1, l) + sweep_steps(H, 2, l);
  for (int i : driven(H)) {
    double* vc = H->h_vtab[(size_t)i * kMaxLevels + l + 1];
    if ((e = fill_launch(vc, (int64_t)(H->Nl[l + 1] + 1) * H->inst[i].ndof, 0.0, st)) != hipSuccess) return e;
  }
  if ((e = level_solve(H, l + 1, kind, st, phi)) != hipSuccess) return e;
  for (int i : driven(H)) {
    double* vl = H->h_vtab[(size_t)i * kMaxLevels + l];
    double* vc = H->h_vtab[(size_t)i * kMaxLevels + l + 1];
    if ((e = correct_launch(vl, vc, H->inst[i].ndof, H->m, H->Nl[l + 1], H->freeze_on ? H->d_frozen + i : nullptr,
                            st)) != hipSuccess)
      return e;
  }
  // ideal interpolation = F-relaxation from the corrected C-points
  phi += sweep_steps(H, 0, l);
  return sweep(H, [l](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jF[l]; }, kModeChain, st);
}

// Approximate solve of the level-l >= 1 problem from its current v (Sec. 3, cycle types): the
// coarsest level by sequential time stepping; otherwise one cycle (kind 0, V), two cycles (kind 1,
// W), or an F-cycle followed by a V-cycle (kind 2, F).
static hipError_t level_solve(pmgrit_handle* H, int l, int kind, hipStream_t st, int64_t& phi) {
  if (l == H->nlev - 1) {
    phi += sweep_steps(H, 3, l);
    return sweep(H, [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jCoarsest; }, kModeChain, st);
  }
  hipError_t e = mgrit_cycle(H, l, kind, st, phi);
  if (e != hipSuccess || kind == 0) return e;
  return mgrit_cycle(H, l, kind == 1 ? 1 : 0, st, phi);
}

static pmgrit_status read_status(pmgrit_handle* H, hipStream_t st) {
  int s[4];
  HIPCHK(hipMemcpyAsync(s, H->d_status, sizeof(s), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (s[0] & 1) return fail(PMGRIT_E_NONFINITE, "non-finite residual in a spatial solve");
  if (s[0] & 2) return fail(PMGRIT_E_SPATIAL_NOCONV, "a spatial solve reached max_vcycles");
  return PMGRIT_OK;
}

static pmgrit_status begin_solve(pmgrit_handle* H, hipStream_t st, double* const* u_out) {
  if (H->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  if (!u_out) return fail(PMGRIT_E_ARG, "u_out_dev is NULL");
  HIPCHK(hipSetDevice(H->device));
  for (int i = 0; i < H->ninst; ++i) {
    if (!u_out[i]) return fail(PMGRIT_E_ARG, "u_out_dev[i] is NULL");
    H->h_vtab[(size_t)i * kMaxLevels] = u_out[i];
  }
  HIPCHK(hipMemcpyAsync(H->d_vtab, H->h_vtab.data(), sizeof(double*) * H->h_vtab.size(), hipMemcpyHostToDevice, st));
  if (H->so.guess == 3) {
    if (!H->net || !H->net->loaded) return fail(PMGRIT_E_STATE, "guess 3 needs a network: call pmgrit_net_load");
    for (int i = 0; i < H->ninst; ++i) {
      H->h_netsrc[i].U = u_out[i];
      H->h_netsrc[i].Uout = u_out[i];
    }
    HIPCHK(hipMemcpyAsync(H->d_netsrc, H->h_netsrc, sizeof(NetSrc) * H->ninst, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemsetAsync(H->d_status, 0, sizeof(int) * 4, st));
  // initial iterate: U_0 = u0, U_k = 0 for k >= 1
  for (int i = 0; i < H->ninst; ++i) {
    const int nd = H->inst[i].ndof;
    HIPCHK(fill_launch(u_out[i] + nd, (int64_t)H->Nt * nd, 0.0, st));
    HIPCHK(hipMemcpyAsync(u_out[i], H->inst[i].u0.data(), sizeof(double) * nd, hipMemcpyHostToDevice, st));
  }
  return PMGRIT_OK;
}

static int64_t sum_vcycles(pmgrit_handle* H, hipStream_t st) {
  int64_t s = 0;
  for (pmgrit_handle::Group& G : H->groups) {
    std::vector<int> v(G.max_jobs);
    if (hipMemcpyAsync(v.data(), G.d_vcount, sizeof(int) * G.max_jobs, hipMemcpyDeviceToHost, st) != hipSuccess)
      return -1;
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    for (int x : v) s += x;
  }
  return s;
}

// Autotuner: for every launch group, time probe solves (level 0 of its first instance, one
// right-hand side per workgroup slot of a level-0 sweep, up to the pmgrit_phi limit) with each LDS
// placement that keeps the triangular-solve vector in LDS, and keep the fastest.  The
// placements differ only in where vectors live, so the arithmetic and the results are the same.
static pmgrit_status autotune(pmgrit_handle* H) {
  HIPCHK(hipSetDevice(H->device));
  const int vt = H->fp32 ? 4 : 8;
  int dev_lds = 0;
  HIPCHK(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, H->device));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (pmgrit_handle::Group& G : H->groups) {
    // groups whose triangular-solve vector is not in LDS (window mode): only the wide (level-0)
    // placement is tuned, between one and two workgroups per CU (FP32)
    const bool window = !(G.mask & kY);
    if (window && (!H->fp32 || H->ext || G.plan.off_win < 0)) continue;
    const int inst = G.inst[0];
    const int nd = H->inst[inst].ndof;
    // two probes: as wide as a level-0 sweep (the wide placement) and as narrow as a level-1
    // sweep (the placement of every narrower launch)
    const int nwide = std::max(1, std::min(kGivenMax, G.jF.empty() ? 64 : std::max(G.jF[0].n, 64)));
    const int nnarrow = std::max(1, std::min(H->ncu, G.jF.size() > 1 ? std::max(G.jF[1].n, 1) : 8));
    const int nrhs = std::max(nwide, nnarrow);
    std::vector<double> hb((size_t)nrhs * nd);
    uint64_t z = 0x2545F4914F6CDD1Dull;
    for (double& v : hb) {  // a fixed pseudo-random right-hand side (xorshift64)
      z ^= z << 13;
      z ^= z >> 7;
      z ^= z << 17;
      v = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    double *b = nullptr, *x = nullptr;
    HIPCHK(hipMalloc(&b, sizeof(double) * hb.size()));
    std::unique_ptr<void, void (*)(void*)> gb(b, [](void* p) { (void)hipFree(p); });
    HIPCHK(hipMalloc(&x, sizeof(double) * hb.size()));
    std::unique_ptr<void, void (*)(void*)> gx(x, [](void* p) { (void)hipFree(p); });
    HIPCHK(hipMemcpy(b, hb.data(), sizeof(double) * hb.size(), hipMemcpyHostToDevice));
    for (int j = 0; j < nrhs; ++j) H->h_given_jobs[j] = PhiJob{inst, 0, 0, 1, 0, 0};
    HIPCHK(hipMemcpy(G.d_given_jobs, H->h_given_jobs, sizeof(PhiJob) * nrhs, hipMemcpyHostToDevice));
    H->given_key[0] = -1;
    // fastest placement for a probe of n right-hand sides
    auto probe = [&](int n, int& best_mask, int& best_bytes, LdsPlan& best_plan, float& best_ms) -> hipError_t {
      best_ms = 1e30f;
      for (int mk : {15, 7, 3, 1, 3 | kOcc2, 1 | kOcc2, 15 | kT1024, 7 | kT1024, 3 | kT1024, 1 | kT1024, 15 | kW8,
                     7 | kW8, 3 | kW8, 1 | kW8, 0, kOcc2}) {
        if (window != ((mk & 15) == 0)) continue;  // window groups: the placements without y in LDS
        if ((mk & kOcc2) && !H->fp32) continue;
        if (H->ext && (mk & (kOcc2 | kT1024 | kW8))) continue;  // the extended build: 512 threads
        mk |= H->ext;
        if ((mk & kW8) && G.maxrows > kRowSlots / 2) continue;
        int bytes = 0;
        const LdsPlan plan = lds_plan_mask(G.nmax, G.n1max, G.maxrows, vt, (mk & (kT1024 | kW8)) ? G.ka8 : G.ka,
                                           dev_lds, G.winw, mk, bytes);
        if (bytes == 0 || ((mk & kOcc2) && 2 * bytes > dev_lds)) continue;
        hipError_t e = phi_prepare(H->fp32, mk, bytes);
        if (e != hipSuccess) return e;
        G.mask = mk;
        G.lds_bytes = bytes;
        G.plan = plan;
        PhiParams P = base_params(H, G, kModeGiven, G.d_given_jobs);
        P.vtab = nullptr;
        P.bgiven = b;
        P.xgiven = x;
        P.guess = 0;
        // the best of three launches after a warm-up one (first-touch and cache effects)
        float ms = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
          float t = 0.f;
          if ((e = hipMemset(x, 0, sizeof(double) * hb.size())) != hipSuccess) return e;
          if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) return e;
          if ((e = phi_launch(H->fp32, mk, bytes, P, plan, n, nullptr)) != hipSuccess) return e;
          if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) return e;
          if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
          if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
          if (rep > 0) ms = std::min(ms, t);
        }
        // the 512-thread build is kept unless another build is at least 3 % faster on the probe
        // (they are often within the probe's noise, and this keeps the choice stable)
        const bool special = mk & (kOcc2 | kT1024 | kW8), best_special = best_mask & (kOcc2 | kT1024 | kW8);
        const float margin = special == best_special ? 1.f : special ? 0.97f : 1.f / 0.97f;
        if (ms < best_ms * margin) {
          best_ms = ms;
          best_mask = mk;
          best_bytes = bytes;
          best_plan = plan;
        }
      }
      return hipSuccess;
    };
    int nm = G.mask, nb = G.lds_bytes, wm = G.mask, wb = G.lds_bytes;
    LdsPlan np = G.plan, wp = G.plan;
    float nms = 0.f, wms = 0.f;
    if (!window) HIPCHK(probe(nnarrow, nm, nb, np, nms));
    if (nwide > H->ncu) {
      HIPCHK(probe(nwide, wm, wb, wp, wms));
    } else {
      wm = nm, wb = nb, wp = np, wms = nms;
    }
    G.mask = nm;
    G.lds_bytes = nb;
    G.plan = np;
    G.wmask = wm;
    G.wbytes = wb;
    G.wplan = wp;
    G.tuned_ms = nms;
    HIPCHK(phi_prepare(H->fp32, G.mask, G.lds_bytes));
    HIPCHK(phi_prepare(H->fp32, G.wmask, G.wbytes));
  }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  HIPCHK(hipMemset(H->d_status, 0, sizeof(int) * 4));
  for (pmgrit_handle::Group& G : H->groups) HIPCHK(hipMemset(G.d_vcount, 0, sizeof(int) * G.max_jobs));
  return PMGRIT_OK;
}

extern "C" {

const char* pmgrit_last_error(void) { return g_err.c_str(); }

pmgrit_status pmgrit_create(int32_t n_instances, const pmgrit_problem* probs, const pmgrit_mgrit_opts* mopts,
                            const pmgrit_solver_opts* sopts, int32_t hip_device, pmgrit_handle** out) {
  auto t0 = std::chrono::steady_clock::now();
  if (!out || !probs || !mopts || !sopts || n_instances < 1) return fail(PMGRIT_E_ARG, "null argument or no instances");
  const pmgrit_mgrit_opts& mo = *mopts;
  const pmgrit_solver_opts& so = *sopts;
  if (mo.cfactor < 2 || mo.max_levels < 1 || mo.max_levels > kMaxLevels || mo.coarsest_max < 1 || mo.max_iter < 0 ||
      !(mo.tol >= 0) || mo.use_graph < 0 || mo.use_graph > 1 || mo.cycle < 0 || mo.cycle > 2)
    return fail(PMGRIT_E_ARG, "invalid MGRIT options");
  if (so.nu1 < 1 || so.nu2 < 0 || !(so.ilut_droptol >= 0) || !(so.spatial_tol > 0) || so.max_vcycles < 1 ||
      (so.precision != 0 && so.precision != 1) || so.guess < 0 || so.guess > 3 || so.trsv_block < -1 ||
      so.autotune < 0 || so.autotune > 1 || !(so.coarse_tol >= 0) || so.coarse_tol >= 1 || so.lds_mask < 0 ||
      so.lds_mask > 127 || (so.lds_mask && so.autotune) ||
      ((so.lds_mask & kT1024) && ((so.lds_mask & kOcc2) || !(so.lds_mask & kY))) ||
      ((so.lds_mask & kW8) && ((so.lds_mask & (kOcc2 | kT1024)) || !(so.lds_mask & kY))) ||
      ((so.lds_mask & kOcc2) && (so.precision != 1 || (so.lds_mask & 15) != ((so.lds_mask & 15) & (kY | kD)) ||
                                 !(so.lds_mask & kY))) ||
      so.solver < 0 || so.solver > 1 || so.coarse < 0 || so.coarse > 1 ||
      // CG runs in FP64 on the 512-thread build
      (so.solver == 1 && (so.precision != 0 || (so.lds_mask & (kOcc2 | kT1024 | kW8)))))
    return fail(PMGRIT_E_ARG, "invalid solver options");
  for (int i = 0; i < n_instances; ++i) {
    const pmgrit_problem& p = probs[i];
    if (p.degree_p < 2 || p.degree_p > 8 || p.n_elems < 2 || p.n_elems > 1024 || (p.domain != 0 && p.domain != 1) ||
        !(p.kappa > 0) || !(p.T > 0) || p.n_steps < 1 || !(p.theta >= 0.0 && p.theta <= 1.0))
      return fail(PMGRIT_E_ARG, "invalid problem " + std::to_string(i));
    if (p.n_steps != probs[0].n_steps) return fail(PMGRIT_E_ARG, "all instances must share n_steps");
  }
  std::unique_ptr<pmgrit_handle> H(new pmgrit_handle());
  H->device = hip_device;
  H->ninst = n_instances;
  for (int i = 0; i < n_instances; ++i) H->all_inst.push_back(i);
  H->mo = mo;
  H->so = so;
  H->Nt = probs[0].n_steps;
  H->m = mo.cfactor;
  // hierarchy: N_l = floor(N_t / m^l) while more than coarsest_max intervals remain
  H->Nl.push_back(H->Nt);
  while ((int)H->Nl.size() < mo.max_levels && H->Nl.back() > mo.coarsest_max && H->Nl.back() / H->m >= 1)
    H->Nl.push_back(H->Nl.back() / H->m);
  H->nlev = (int)H->Nl.size();
  H->inst.resize(n_instances);
  {
    std::string err;
    pmgrit_status st = parallel_tasks(
        n_instances,
        [&](int i, std::string& e) {
          pmgrit_status r = setup_instance(H.get(), H->inst[i], probs[i]);
          if (r != PMGRIT_OK) e = "p=1 mass matrix of instance " + std::to_string(i) + " is not SPD";
          return r;
        },
        err);
    if (st != PMGRIT_OK) return fail(st, err);
    st = parallel_tasks(
        n_instances * H->nlev,
        [&](int t, std::string& e) { return setup_level(H.get(), H->inst[t / H->nlev], t % H->nlev, e); }, err);
    if (st != PMGRIT_OK) return fail(st, err);
  }
  if (hip_device >= 0) {
    pmgrit_status s = device_setup(H.get());
    if (s == PMGRIT_OK && H->so.autotune) s = autotune(H.get());
    if (s != PMGRIT_OK) {
      std::string keep = g_err;
      pmgrit_destroy(H.release());
      g_err = keep;
      return s;
    }
  }
  H->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = H.release();
  return PMGRIT_OK;
}

void pmgrit_destroy(pmgrit_handle* h) {
  if (!h) return;
  if (h->device >= 0) {
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (void* p : h->allocs) (void)hipFree(p);
    if (h->h_pinned) (void)hipHostFree(h->h_pinned);
    if (h->h_frozen) (void)hipHostFree(h->h_frozen);
    if (h->h_given_jobs) (void)hipHostFree(h->h_given_jobs);
    if (h->h_netsrc) (void)hipHostFree(h->h_netsrc);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    if (h->gfork) (void)hipEventDestroy(h->gfork);
    if (h->gjoin) (void)hipEventDestroy(h->gjoin);
    h->net.reset();
    for (hipEvent_t e : h->ev)
      if (e) (void)hipEventDestroy(e);
    for (pmgrit_handle::Group& G : h->groups) {
      if (G.done) (void)hipEventDestroy(G.done);
      if (G.stream) (void)hipStreamDestroy(G.stream);
    }
    if (h->fork) (void)hipEventDestroy(h->fork);
  }
  delete h;
}

pmgrit_status pmgrit_dims(const pmgrit_handle* h, int32_t inst, int64_t* n_dof, int32_t* grid_n, int32_t* n_levels) {
  if (!h || inst < 0 || inst >= h->ninst) return fail(PMGRIT_E_ARG, "bad handle or instance");
  if (n_dof) *n_dof = h->inst[inst].ndof;
  if (grid_n) *grid_n = h->inst[inst].N;
  if (n_levels) *n_levels = h->nlev;
  return PMGRIT_OK;
}

static std::vector<double> modal_load(const InstHost& I, int nm, const int32_t* k, const int32_t* l, const double* a) {
  const bool ann = I.domain == 1;
  std::vector<double> out(I.ndof, 0.0);
  for (int q = 0; q < nm; ++q) {
    std::vector<double> fx = mode_load_1d(I.n, I.p, k[q], ann ? 1 : 0, I.p + 1);
    std::vector<double> fy = mode_load_1d(I.n, I.p, l[q], ann ? 3 : 0, I.p + 1);
    for (int iy = 1; iy <= I.Nin; ++iy)
      for (int ix = 1; ix <= I.Nin; ++ix) out[(size_t)(iy - 1) * I.Nin + (ix - 1)] += a[q] * fx[ix] * fy[iy];
  }
  return out;
}

pmgrit_status pmgrit_set_source_modes(pmgrit_handle* h, int32_t inst, int32_t n_modes, const int32_t* k,
                                      const int32_t* l, const double* amp, int32_t time_kind) {
  if (!h || inst < 0 || inst >= h->ninst || n_modes < 0 || (n_modes > 0 && (!k || !l || !amp)) ||
      (time_kind != 0 && time_kind != 1))
    return fail(PMGRIT_E_ARG, "bad source arguments");
  InstHost& I = h->inst[inst];
  for (int q = 0; q < n_modes; ++q)
    if (k[q] < 0 || l[q] < 0) return fail(PMGRIT_E_ARG, "negative mode number");
  I.F = modal_load(I, n_modes, k, l, amp);
  I.tkind = time_kind;
  const double dt = I.prob.T / I.prob.n_steps;
  // source weight of step s - 1 -> s, theta-weighted like the diffusion term:
  // w = dt (theta tfac(t_s) + (1 - theta) tfac(t_{s-1})); entry 0 is dt tfac(0)
  auto tf = [&](int s) { return time_kind == 1 ? std::exp(-s * dt) : 1.0; };
  const double th = I.prob.theta;
  I.scale[0] = dt * tf(0);
  for (int s = 1; s <= I.prob.n_steps; ++s) I.scale[s] = dt * (th * tf(s) + (1.0 - th) * tf(s - 1));
  if (h->device >= 0) {
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipMemcpy((void*)h->h_instdev[inst].F, I.F.data(), sizeof(double) * I.ndof, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy((void*)h->h_instdev[inst].scale, I.scale.data(), sizeof(double) * I.scale.size(),
                     hipMemcpyHostToDevice));
  }
  return PMGRIT_OK;
}

pmgrit_status pmgrit_set_initial_modes(pmgrit_handle* h, int32_t inst, int32_t n_modes, const int32_t* k,
                                       const int32_t* l, const double* amp) {
  if (!h || inst < 0 || inst >= h->ninst || n_modes < 0 || (n_modes > 0 && (!k || !l || !amp)))
    return fail(PMGRIT_E_ARG, "bad initial-condition arguments");
  InstHost& I = h->inst[inst];
  if (n_modes == 0) {
    I.u0.assign(I.ndof, 0.0);
    return PMGRIT_OK;
  }
  // L2 projection: solve M c = int u0 Phi by conjugate gradients with Jacobi preconditioning
  std::vector<double> b = modal_load(I, n_modes, k, l, amp), x(I.ndof, 0.0), r = b, z(I.ndof), pdir(I.ndof),
                      Ap(I.ndof), dg(I.ndof);
  const Csr& M = I.M;
  for (int i = 0; i < I.ndof; ++i)
    for (int t = M.rp[i]; t < M.rp[i + 1]; ++t)
      if (M.ci[t] == i) dg[i] = M.v[t];
  auto dot = [](const std::vector<double>& a, const std::vector<double>& c) {
    double s = 0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * c[i];
    return s;
  };
  for (int i = 0; i < I.ndof; ++i) z[i] = r[i] / dg[i];
  pdir = z;
  double rz = dot(r, z), bn = std::sqrt(dot(b, b));
  for (int it = 0; it < 20000 && std::sqrt(dot(r, r)) > 1e-15 * bn; ++it) {
    for (int i = 0; i < I.ndof; ++i) {
      double s = 0;
      for (int t = M.rp[i]; t < M.rp[i + 1]; ++t) s += M.v[t] * pdir[M.ci[t]];
      Ap[i] = s;
    }
    double alpha = rz / dot(pdir, Ap);
    for (int i = 0; i < I.ndof; ++i) {
      x[i] += alpha * pdir[i];
      r[i] -= alpha * Ap[i];
      z[i] = r[i] / dg[i];
    }
    double rz2 = dot(r, z);
    for (int i = 0; i < I.ndof; ++i) pdir[i] = z[i] + rz2 / rz * pdir[i];
    rz = rz2;
  }
  I.u0 = x;
  return PMGRIT_OK;
}

pmgrit_status pmgrit_set_initial_coeffs(pmgrit_handle* h, int32_t inst, const double* u0_host) {
  if (!h || inst < 0 || inst >= h->ninst || !u0_host) return fail(PMGRIT_E_ARG, "bad initial coefficients");
  InstHost& I = h->inst[inst];
  I.u0.assign(u0_host, u0_host + I.ndof);
  return PMGRIT_OK;
}

// level-0 F-relaxation, C-relaxation with the following F-relaxation, C-point residuals and their
// norms per instance (into d_resnorm)
static hipError_t relax_level0(pmgrit_handle* h, hipStream_t st, bool learned, int64_t& phi) {
  hipError_t e;
  if (learned) {
    // learned guesses: the same relaxations one step position at a time, each preceded by the
    // network's predictions for its targets
    auto fsplit = [&]() -> hipError_t {
      for (int s = 0; s + 1 < h->m; ++s) {
        hipError_t e2 = net_predict(h, 1, s, 0, st);
        if (e2 == hipSuccess)
          e2 = sweep(h, [s](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jF1[s]; }, kModeChain, st,
                     4);
        if (e2 != hipSuccess) return e2;
      }
      return hipSuccess;
    };
    if ((e = fsplit()) != hipSuccess) return e;
    if ((e = net_predict(h, 2, 0, 0, st)) != hipSuccess) return e;
    if ((e = sweep(h, [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jC1; }, kModeChain, st, 4)) !=
        hipSuccess)
      return e;
    if ((e = fsplit()) != hipSuccess) return e;
  } else {
    auto f0 = [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jF[0]; };
    if ((e = sweep(h, f0, kModeChain, st)) != hipSuccess) return e;
    if ((e = sweep(h, [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jC[0]; }, kModeChain, st)) !=
        hipSuccess)
      return e;
    if ((e = sweep(h, f0, kModeChain, st)) != hipSuccess) return e;
  }
  if ((e = sweep(h, [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jRES[0]; }, kModeResidual,
                 st)) != hipSuccess)
    return e;
  for (int gi = 0; gi < (int)h->groups.size(); ++gi) {
    if (!drives(h, gi)) continue;
    pmgrit_handle::Group& G = h->groups[gi];
    if ((e = norm_reduce_launch(G.d_nrm2, G.d_res_begin, G.d_res_inst, h->d_resnorm, (int)G.inst.size(), st)) !=
        hipSuccess)
      return e;
  }
  phi += 2 * sweep_steps(h, 0, 0) + sweep_steps(h, 1, 0) + sweep_steps(h, 2, 0);
  return hipSuccess;
}

// coarse-grid correction of level 0: solve the level-1 correction equation by a recursive cycle
// and add it to the level-0 C-points
static hipError_t correct_level0(pmgrit_handle* h, hipStream_t st, double* const* u_out, int64_t& phi) {
  hipError_t e;
  for (int i : driven(h)) {
    double* vc = h->h_vtab[(size_t)i * kMaxLevels + 1];
    if ((e = fill_launch(vc, (int64_t)(h->Nl[1] + 1) * h->inst[i].ndof, 0.0, st)) != hipSuccess) return e;
  }
  if ((e = level_solve(h, 1, h->mo.cycle, st, phi)) != hipSuccess) return e;
  for (int i : driven(h)) {
    double* vc = h->h_vtab[(size_t)i * kMaxLevels + 1];
    if ((e = correct_launch(u_out[i], vc, h->inst[i].ndof, h->m, h->Nl[1], h->freeze_on ? h->d_frozen + i : nullptr,
                            st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// one MGRIT iteration after the first: the coarse-grid correction, then the next level-0
// relaxation. With several launch groups each group runs its whole iteration on its own stream
// (groups share no vectors, scratch or job lists), so a group with short sweeps goes on to its
// level-0 sweeps while a larger group is still in its narrow coarse-level sweeps, rather than all
// groups meeting after every sweep.
static hipError_t mgrit_iteration(pmgrit_handle* h, hipStream_t st, double* const* u_out, int64_t& phi) {
  hipError_t e;
  if (h->groups.size() == 1) {
    if ((e = correct_level0(h, st, u_out, phi)) != hipSuccess) return e;
    return relax_level0(h, st, false, phi);
  }
  if ((e = hipEventRecord(h->fork, st)) != hipSuccess) return e;
  for (int gi : h->launch_order) {
    pmgrit_handle::Group& G = h->groups[gi];
    if ((e = hipStreamWaitEvent(G.stream, h->fork, 0)) != hipSuccess) return e;
    h->only_group = gi;
    e = correct_level0(h, G.stream, u_out, phi);
    if (e == hipSuccess) e = relax_level0(h, G.stream, false, phi);
    h->only_group = -1;
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(G.done, G.stream)) != hipSuccess) return e;
  }
  for (pmgrit_handle::Group& G : h->groups)
    if ((e = hipStreamWaitEvent(st, G.done, 0)) != hipSuccess) return e;
  return hipSuccess;
}

// The first level-0 relaxation. Without the learned guess every group relaxes whole on its own
// stream, as in the later iterations. With it, the groups holding an instance the network predicts
// go step position by position, joined at every sweep (one position's predictions span those
// groups), while every other group relaxes whole on its own stream meanwhile.
static hipError_t relax_first(pmgrit_handle* h, hipStream_t st, bool learned, int64_t& phi) {
  if (h->groups.size() == 1) return relax_level0(h, st, learned, phi);
  hipError_t e;
  if ((e = hipEventRecord(h->fork, st)) != hipSuccess) return e;
  bool any_net = false;
  for (int gi : h->launch_order) {
    pmgrit_handle::Group& G = h->groups[gi];
    if (learned && !G.netfree) {
      any_net = true;
      continue;
    }
    if ((e = hipStreamWaitEvent(G.stream, h->fork, 0)) != hipSuccess) return e;
    h->only_group = gi;
    e = relax_level0(h, G.stream, false, phi);
    h->only_group = -1;
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(G.done, G.stream)) != hipSuccess) return e;
  }
  if (any_net) {
    h->skip_netfree = true;
    e = relax_level0(h, st, true, phi);
    h->skip_netfree = false;
    if (e != hipSuccess) return e;
  }
  for (pmgrit_handle::Group& G : h->groups)
    if ((!learned || G.netfree) && (e = hipStreamWaitEvent(st, G.done, 0)) != hipSuccess) return e;
  return hipSuccess;
}

// one MGRIT iteration after the first (correction, then the next relaxation) captured as a HIP
// graph for the given trajectory buffers; the kernels only (no memset or copy nodes)
static pmgrit_status capture_iteration(pmgrit_handle* h, hipStream_t st, double* const* u_out) {
  std::vector<void*> key(u_out, u_out + h->ninst);
  if (h->graph_exec && key == h->graph_key && h->graph_stream == st) return PMGRIT_OK;
  if (h->graph_exec) {
    HIPCHK(hipGraphExecDestroy(h->graph_exec));
    h->graph_exec = nullptr;
  }
  const bool prof = h->prof;
  h->prof = false;  // no timing events inside the graph
  hipGraph_t g = nullptr;
  int64_t phi = 0;
  const int64_t nl0 = h->nlaunch_total, nw0 = h->nwg_total;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t eb = mgrit_iteration(h, st, u_out, phi);
    e = hipStreamEndCapture(st, &g);
    if (eb != hipSuccess) e = eb;
  }
  h->prof = prof;
  if (e == hipSuccess) e = hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph_exec = nullptr;
    return fail(PMGRIT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  h->graph_key = key;
  h->graph_stream = st;
  h->graph_phi = phi;
  h->graph_launches = h->nlaunch_total - nl0;
  h->graph_wgs = h->nwg_total - nw0;
  h->nlaunch_total = nl0;
  h->nwg_total = nw0;
  return PMGRIT_OK;
}

// replay of the captured iteration; with timing on, one event pair brackets the whole graph (its
// spatial-solve launches are counted, the small kernels between them are included in the time)
static hipError_t graph_launch_timed(pmgrit_handle* h, hipStream_t st) {
  h->nlaunch_total += h->graph_launches;
  h->nwg_total += h->graph_wgs;
  if (!h->prof) return hipGraphLaunch(h->graph_exec, st);
  hipError_t e;
  if (h->ev_used * 2 + 2 > (int)h->ev.size()) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    if ((e = harvest(h)) != hipSuccess) return e;
  }
  const int k = h->ev_used++;
  h->ev_group[k] = -1;
  if ((e = hipEventRecord(h->ev[2 * k], st)) != hipSuccess) return e;
  if ((e = hipGraphLaunch(h->graph_exec, st)) != hipSuccess) return e;
  h->prof_launches += h->graph_launches;
  h->prof_wgs += h->graph_wgs;
  return hipEventRecord(h->ev[2 * k + 1], st);
}

pmgrit_status pmgrit_solve_mgrit(pmgrit_handle* h, void* hip_stream, double* const* u_out_dev, pmgrit_stats* stats) {
  if (!h) return fail(PMGRIT_E_ARG, "null handle");
  hipStream_t st = (hipStream_t)hip_stream;
  auto t0 = std::chrono::steady_clock::now();
  TRY(begin_solve(h, st, u_out_dev));
  const int64_t vc0 = sum_vcycles(h, st);
  pmgrit_stats S;
  std::memset(&S, 0, sizeof(S));
  int64_t phi = 0;
  int iters = 0;
  pmgrit_status rc = PMGRIT_OK;
  hipStream_t caller = nullptr;
  bool forked = false;
  auto seq = [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jSeq; };
  if (h->nlev == 1) {
    HIPCHK(sweep(h, seq, kModeChain, st, h->so.guess == 0 ? 0 : 1));
    phi += sweep_steps(h, 4, 0);
  } else {
    const bool graph = h->mo.use_graph != 0;
    // an instance whose residual reaches the tolerance keeps that iterate: from the next
    // iteration on, its jobs and corrections are skipped (the flags are read at replay, so the
    // captured graph holds the flag array too)
    h->freeze_on = true;
    struct Unfreeze {
      pmgrit_handle* h;
      ~Unfreeze() { h->freeze_on = false; }
    } unfreeze{h};  // every exit, the error returns included, leaves the other entry points unaffected
    if (graph) {
      // the whole solve runs on the library's own stream, ordered after the caller's work
      HIPCHK(hipEventRecord(h->gfork, st));
      HIPCHK(hipStreamWaitEvent(h->gstream, h->gfork, 0));
      caller = st;
      st = h->gstream;
      forked = true;
      TRY(capture_iteration(h, st, u_out_dev));
    }
    std::vector<double> r0(h->ninst, -1.0), rfix(h->ninst, 0.0);
    std::memset(h->h_frozen, 0, sizeof(int) * h->ninst);
    HIPCHK(hipMemcpyAsync(h->d_frozen, h->h_frozen, sizeof(int) * h->ninst, hipMemcpyHostToDevice, st));
    HIPCHK(relax_first(h, st, h->so.guess == 3, phi));
    for (;;) {
      HIPCHK(hipMemcpyAsync(h->h_pinned, h->d_resnorm, sizeof(double) * h->ninst, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(harvest(h));
      bool done = true, bad = false, newly = false;
      double worst = 0.0;
      for (int i = 0; i < h->ninst; ++i) {
        if (h->h_frozen[i]) {
          // no residual was computed for it: its value at freezing stands
          worst = std::max(worst, rfix[i]);
          continue;
        }
        double rn = std::sqrt(h->h_pinned[i]);
        if (!std::isfinite(rn)) bad = true;
        if (r0[i] < 0) r0[i] = rn;
        double rel = r0[i] > 0 ? rn / r0[i] : 0.0;
        worst = std::max(worst, rel);
        if (rn <= h->mo.tol * r0[i] || r0[i] == 0.0) {
          h->h_frozen[i] = 1;
          rfix[i] = rel;
          newly = true;
        } else {
          done = false;
        }
      }
      if (iters < 64) S.res_hist[iters] = worst;
      pmgrit_status s = read_status(h, st);
      if (s != PMGRIT_OK) {
        rc = s;
        break;
      }
      if (bad) {
        rc = fail(PMGRIT_E_NONFINITE, "non-finite MGRIT residual");
        break;
      }
      if (done) break;
      if (iters >= h->mo.max_iter) {
        rc = fail(PMGRIT_E_MGRIT_NOCONV, "MGRIT reached max_iter");
        break;
      }
      if (newly)
        HIPCHK(hipMemcpyAsync(h->d_frozen, h->h_frozen, sizeof(int) * h->ninst, hipMemcpyHostToDevice, st));
      // every instance has the same N_t, so it takes the same share of every sweep's solves;
      // frozen instances take none
      int64_t it_phi = 0;
      if (graph) {
        HIPCHK(graph_launch_timed(h, st));
        it_phi = h->graph_phi;
      } else {
        HIPCHK(mgrit_iteration(h, st, u_out_dev, it_phi));
      }
      int active = 0;
      for (int i = 0; i < h->ninst; ++i) active += h->h_frozen[i] ? 0 : 1;
      phi += it_phi / h->ninst * active;
      ++iters;
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  if (forked) {
    HIPCHK(hipEventRecord(h->gjoin, st));
    HIPCHK(hipStreamWaitEvent(caller, h->gjoin, 0));
  }
  HIPCHK(harvest(h));
  if (rc == PMGRIT_OK) rc = read_status(h, st);
  S.mgrit_iters = iters;
  S.phi_calls = phi;
  S.vcycles = sum_vcycles(h, st) - vc0;
  S.t_setup_s = h->t_setup;
  S.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = S;
  return rc;
}

pmgrit_status pmgrit_solve_sequential(pmgrit_handle* h, void* hip_stream, double* const* u_out_dev,
                                      pmgrit_stats* stats) {
  if (!h) return fail(PMGRIT_E_ARG, "null handle");
  hipStream_t st = (hipStream_t)hip_stream;
  auto t0 = std::chrono::steady_clock::now();
  TRY(begin_solve(h, st, u_out_dev));
  const int64_t vc0 = sum_vcycles(h, st);
  if (h->so.guess == 3) {
    // one launch per step: predictions, then the solves starting from the better of the
    // prediction and the previous point
    for (int k = 0; k < h->Nt; ++k) {
      HIPCHK(net_predict(h, 0, 0, k, st));
      HIPCHK(sweep(h, [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jSeq1; }, kModeChain, st, 4,
                   k));
    }
  } else {
    HIPCHK(sweep(h, [](pmgrit_handle::Group& G) -> pmgrit_handle::JobList& { return G.jSeq; }, kModeChain, st,
                 h->so.guess == 0 ? 0 : 1));
  }
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(harvest(h));
  pmgrit_status rc = read_status(h, st);
  if (stats) {
    pmgrit_stats S;
    std::memset(&S, 0, sizeof(S));
    S.phi_calls = sweep_steps(h, 4, 0);
    S.vcycles = sum_vcycles(h, st) - vc0;
    S.t_setup_s = h->t_setup;
    S.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *stats = S;
  }
  return rc;
}

pmgrit_status pmgrit_phi(pmgrit_handle* h, int32_t inst, int32_t level, int32_t nrhs, const double* b_dev,
                         double* x_dev, int32_t* vcycles_dev, void* hip_stream) {
  if (!h || inst < 0 || inst >= h->ninst || level < 0 || level >= h->nlev || nrhs < 0 || nrhs > kGivenMax ||
      (nrhs > 0 && (!b_dev || !x_dev)))
    return fail(PMGRIT_E_ARG, "bad pmgrit_phi arguments");
  if (h->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  if (nrhs == 0) return PMGRIT_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  HIPCHK(hipSetDevice(h->device));
  pmgrit_handle::Group& G = h->groups[h->inst_group[inst]];
  if (h->given_key[0] != inst || h->given_key[1] != level || h->given_key[2] < nrhs) {
    // the pinned staging buffer may still feed an earlier copy: wait before rewriting it
    HIPCHK(hipDeviceSynchronize());
    for (int j = 0; j < nrhs; ++j) h->h_given_jobs[j] = PhiJob{inst, level, 0, 1, 0, 0};
    HIPCHK(hipMemcpyAsync(G.d_given_jobs, h->h_given_jobs, sizeof(PhiJob) * nrhs, hipMemcpyHostToDevice, st));
    h->given_key[0] = inst;
    h->given_key[1] = level;
    h->given_key[2] = nrhs;
  }
  PhiParams P = base_params(h, G, kModeGiven, G.d_given_jobs);
  P.vtab = nullptr;
  P.bgiven = b_dev;
  P.xgiven = x_dev;
  P.vlast = vcycles_dev;
  HIPCHK(phi_timed(h, G, P, nrhs, st));
  return PMGRIT_OK;
}

pmgrit_status pmgrit_phi_noalloc(pmgrit_handle* h, int32_t inst, int32_t level, int32_t nrhs, const double* b_dev,
                                 double* x_dev, int32_t* vcycles_dev, void* hip_stream) {
  if (!h || inst < 0 || inst >= h->ninst || level < 0 || level >= h->nlev || nrhs < 0 || nrhs > kGivenMax ||
      (nrhs > 0 && (!b_dev || !x_dev)))
    return fail(PMGRIT_E_ARG, "bad pmgrit_phi_noalloc arguments");
  if (h->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  if (nrhs == 0) return PMGRIT_OK;
  pmgrit_handle::Group& G = h->groups[h->inst_group[inst]];
  if ((int64_t)nrhs * G.ws_stride > kScratchDoubles)
    return fail(PMGRIT_E_ARG, "pmgrit_phi_noalloc: nrhs * " + std::to_string(G.ws_stride) +
                                  " scratch doubles exceed the fixed scratch of " + std::to_string(kScratchDoubles));
  double* ws = scratch_ptr(h->device);
  if (!ws) return fail(PMGRIT_E_STATE, "fixed scratch not set up on this device");
  hipStream_t st = (hipStream_t)hip_stream;
  HIPCHK(hipSetDevice(h->device));
  if (h->given_key[0] != inst || h->given_key[1] != level || h->given_key[2] < nrhs) {
    // the pinned staging buffer may still feed an earlier copy: wait before rewriting it
    HIPCHK(hipDeviceSynchronize());
    for (int j = 0; j < nrhs; ++j) h->h_given_jobs[j] = PhiJob{inst, level, 0, 1, 0, 0};
    HIPCHK(hipMemcpyAsync(G.d_given_jobs, h->h_given_jobs, sizeof(PhiJob) * nrhs, hipMemcpyHostToDevice, st));
    h->given_key[0] = inst;
    h->given_key[1] = level;
    h->given_key[2] = nrhs;
  }
  PhiParams P = base_params(h, G, kModeGiven, G.d_given_jobs);
  P.vtab = nullptr;
  P.bgiven = b_dev;
  P.xgiven = x_dev;
  P.vlast = vcycles_dev;
  P.ws = ws;  // the per-workgroup slices live in the fixed scratch instead of the handle's buffer
  HIPCHK(phi_timed(h, G, P, nrhs, st));
  return PMGRIT_OK;
}

pmgrit_status pmgrit_host_matrix(const pmgrit_handle* h, int32_t inst, int32_t level, int32_t which, int32_t* shape3,
                                 int32_t* rp, int32_t* ci, double* v) {
  if (!h || inst < 0 || inst >= h->ninst || level < 0 || level >= h->nlev || !shape3)
    return fail(PMGRIT_E_ARG, "bad inspection arguments");
  const InstHost& I = h->inst[inst];
  const Csr* A = nullptr;
  switch (which) {
    case 0: A = &I.M; break;
    case 1: A = &I.K; break;
    case 2: A = &I.lev[level].A; break;
    case 3: A = &I.lev[level].L; break;
    case 4: A = &I.lev[level].U; break;
    case 5: A = &I.P; break;
    case 6: A = &I.M1; break;
    case 7: A = &I.K1; break;
    default: return fail(PMGRIT_E_ARG, "bad matrix selector");
  }
  shape3[0] = A->nr;
  shape3[1] = A->nc;
  shape3[2] = A->nnz();
  if (rp) {
    if (!ci || !v) return fail(PMGRIT_E_ARG, "null output array");
    std::memcpy(rp, A->rp.data(), sizeof(int) * (A->nr + 1));
    std::memcpy(ci, A->ci.data(), sizeof(int) * A->nnz());
    std::memcpy(v, A->v.data(), sizeof(double) * A->nnz());
  }
  return PMGRIT_OK;
}

pmgrit_status pmgrit_host_vectors(const pmgrit_handle* h, int32_t inst, double* mlp, double* ml1, double* load,
                                  double* u0) {
  if (!h || inst < 0 || inst >= h->ninst) return fail(PMGRIT_E_ARG, "bad inspection arguments");
  const InstHost& I = h->inst[inst];
  if (mlp) std::memcpy(mlp, I.mlp.data(), sizeof(double) * I.ndof);
  if (ml1) std::memcpy(ml1, I.ml1.data(), sizeof(double) * I.ndof1);
  if (load) std::memcpy(load, I.F.data(), sizeof(double) * I.ndof);
  if (u0) std::memcpy(u0, I.u0.data(), sizeof(double) * I.ndof);
  return PMGRIT_OK;
}

pmgrit_status pmgrit_host_schedule(const pmgrit_handle* h, int32_t inst, int32_t level, int32_t factor, int32_t* out4) {
  if (!h || inst < 0 || inst >= h->ninst || level < 0 || level >= h->nlev || (factor != 0 && factor != 1) || !out4)
    return fail(PMGRIT_E_ARG, "bad inspection arguments");
  const TriSchedule& S = factor == 0 ? h->inst[inst].lev[level].SL : h->inst[inst].lev[level].SU;
  out4[0] = S.nlev;
  out4[1] = S.nblocks;
  out4[2] = S.bs;
  out4[3] = S.max_rows;
  return PMGRIT_OK;
}

pmgrit_status pmgrit_host_coarse_solve(const pmgrit_handle* h, int32_t inst, int32_t level, const double* b,
                                       double* x) {
  if (!h || inst < 0 || inst >= h->ninst || level < 0 || level >= h->nlev || !b || !x)
    return fail(PMGRIT_E_ARG, "bad inspection arguments");
  host_coarse_solve(h->inst[inst], level, b, x);
  return PMGRIT_OK;
}

pmgrit_status pmgrit_profile(pmgrit_handle* h, int32_t enable, double* out4) {
  if (!h || enable < -1 || enable > 1) return fail(PMGRIT_E_ARG, "bad profile arguments");
  if (h->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  HIPCHK(hipSetDevice(h->device));
  if (out4 || enable >= 0) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(harvest(h));
  }
  const int64_t vc = sum_vcycles(h, nullptr);
  if (vc < 0) return fail(PMGRIT_E_HIP, "reading V-cycle counters failed");
  if (out4) {
    out4[0] = h->prof_ms;
    out4[1] = (double)h->prof_launches;
    out4[2] = (double)h->prof_wgs;
    out4[3] = (double)(vc - h->vc_base);
  }
  if (enable == 1) {
    h->prof_ms = 0;
    h->prof_launches = h->prof_wgs = 0;
    h->vc_base = vc;
    std::fill(h->gprof_ms.begin(), h->gprof_ms.end(), 0.0);
    std::fill(h->gprof_launches.begin(), h->gprof_launches.end(), 0);
    std::fill(h->gprof_wgs.begin(), h->gprof_wgs.end(), 0);
  }
  if (enable >= 0) h->prof = enable == 1;
  return PMGRIT_OK;
}

pmgrit_status pmgrit_group_profile(pmgrit_handle* h, int32_t group, double* out3) {
  if (!h || !out3) return fail(PMGRIT_E_ARG, "bad group-profile arguments");
  if (h->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  if (group < 0 || group >= (int)h->groups.size()) return fail(PMGRIT_E_ARG, "bad launch group");
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(harvest(h));
  out3[0] = h->gprof_ms[group];
  out3[1] = (double)h->gprof_launches[group];
  out3[2] = (double)h->gprof_wgs[group];
  return PMGRIT_OK;
}

pmgrit_status pmgrit_inst_vcycles(pmgrit_handle* h, int64_t* out) {
  if (!h || !out) return fail(PMGRIT_E_ARG, "bad counter arguments");
  if (h->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  HIPCHK(hipSetDevice(h->device));
  std::vector<unsigned long long> v(h->ninst);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(v.data(), h->d_vinst, sizeof(unsigned long long) * h->ninst, hipMemcpyDeviceToHost));
  for (int i = 0; i < h->ninst; ++i) out[i] = (int64_t)v[i];
  return PMGRIT_OK;
}

pmgrit_status pmgrit_info(const pmgrit_handle* h, int64_t* out8) {
  if (!h || !out8) return fail(PMGRIT_E_ARG, "bad info arguments");
  int dev_lds = 0;
  if (h->device >= 0) (void)hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
  // launch configuration of the first (largest-LDS) group
  const bool g = !h->groups.empty();
  out8[0] = h->so.precision;
  out8[1] = g ? h->groups[0].mask : -1;
  out8[2] = g ? h->groups[0].lds_bytes : 0;
  out8[3] = dev_lds;
  out8[4] = g ? h->groups[0].ws_stride : 0;
  out8[5] = g ? h->groups[0].max_jobs : 0;
  out8[6] = h->nlev;
  out8[7] = h->ninst;
  return PMGRIT_OK;
}

pmgrit_status pmgrit_group_info(const pmgrit_handle* h, int32_t inst, int64_t* out8) {
  if (!h || !out8 || inst < 0 || inst >= h->ninst) return fail(PMGRIT_E_ARG, "bad group-info arguments");
  if (h->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  const pmgrit_handle::Group& G = h->groups[h->inst_group[inst]];
  out8[0] = h->inst_group[inst];
  out8[1] = (int64_t)h->groups.size();
  out8[2] = G.mask | (G.wmask << 8);
  out8[3] = G.lds_bytes;
  out8[4] = G.ka;
  out8[5] = (int64_t)G.inst.size();
  out8[6] = G.nmax;
  out8[7] = G.max_jobs;
  return PMGRIT_OK;
}

static pmgrit_status net_ready(pmgrit_handle* h) {
  if (h->device < 0) return fail(PMGRIT_E_STATE, "host-only handle");
  HIPCHK(hipSetDevice(h->device));
  if (!h->net) {
    std::unique_ptr<NetState> n(new NetState());
    HIPCHK(n->init(h->device));
    h->net = std::move(n);
  }
  return PMGRIT_OK;
}

int64_t pmgrit_net_nparams(void) { return kNetParams; }

pmgrit_status pmgrit_net_load(pmgrit_handle* h, const float* weights_host, int64_t n) {
  if (!h || !weights_host || n != kNetParams) return fail(PMGRIT_E_ARG, "bad network parameters");
  TRY(net_ready(h));
  HIPCHK(h->net->load(weights_host));
  // buffers for the solve paths' batches, so solving allocates nothing
  for (const pmgrit_handle::NetGroup& N : h->ngroups) {
    int nb = std::max((int)N.inst.size(), N.nc);
    for (int x : N.nf) nb = std::max(nb, x);
    HIPCHK(h->net->reserve(nb, N.G));
  }
  return PMGRIT_OK;
}

pmgrit_status pmgrit_net_save(const pmgrit_handle* h, float* weights_host, int64_t n) {
  if (!h || !weights_host || n != kNetParams) return fail(PMGRIT_E_ARG, "bad network parameters");
  if (h->device < 0 || !h->net || !h->net->loaded) return fail(PMGRIT_E_STATE, "no network loaded");
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(h->net->save(weights_host));
  return PMGRIT_OK;
}

static pmgrit_status net_args(pmgrit_handle* h, int32_t G, int32_t nb, const void* x, const void* y) {
  if (!h || G < 3 || G > 1024 || nb < 1 || !x || !y) return fail(PMGRIT_E_ARG, "bad network arguments");
  TRY(net_ready(h));
  if (!h->net->loaded) return fail(PMGRIT_E_STATE, "no network loaded");
  return PMGRIT_OK;
}

pmgrit_status pmgrit_net_forward(pmgrit_handle* h, int32_t G, int32_t nb, const float* x_dev, float* y_dev,
                                 void* hip_stream) {
  TRY(net_args(h, G, nb, x_dev, y_dev));
  HIPCHK(h->net->forward(nb, G, x_dev, y_dev, (hipStream_t)hip_stream));
  return PMGRIT_OK;
}

pmgrit_status pmgrit_net_grad(pmgrit_handle* h, int32_t G, int32_t nb, const float* x_dev, const float* t_dev,
                              float* grad_host, double* loss_host, void* hip_stream) {
  TRY(net_args(h, G, nb, x_dev, t_dev));
  HIPCHK(h->net->loss_and_grad(nb, G, x_dev, t_dev, grad_host, loss_host, (hipStream_t)hip_stream));
  return PMGRIT_OK;
}

pmgrit_status pmgrit_net_train_step(pmgrit_handle* h, int32_t G, int32_t nb, const float* x_dev, const float* t_dev,
                                    float lr, double* loss_host, void* hip_stream) {
  TRY(net_args(h, G, nb, x_dev, t_dev));
  if (!(lr >= 0.f)) return fail(PMGRIT_E_ARG, "bad learning rate");
  hipStream_t st = (hipStream_t)hip_stream;
  HIPCHK(h->net->backward(nb, G, x_dev, t_dev, st));
  HIPCHK(h->net->adam_step(lr, st));
  if (loss_host) HIPCHK(h->net->read_loss(loss_host, st));
  HIPCHK(hipStreamSynchronize(st));
  return PMGRIT_OK;
}

pmgrit_status pmgrit_net_pack(pmgrit_handle* h, int32_t inst, int32_t level, int32_t nb, const int32_t* k_host,
                              const double* U_dev, float* x_dev, float* t_dev, double* s_dev, void* hip_stream) {
  if (!h || inst < 0 || inst >= h->ninst || level < 0 || level >= h->nlev || nb < 1 || nb > kGivenMax || !k_host ||
      !U_dev || !x_dev || !s_dev)
    return fail(PMGRIT_E_ARG, "bad pack arguments");
  const int lim = h->Nl[level] - (t_dev ? 1 : 0);
  for (int j = 0; j < nb; ++j)
    if (k_host[j] < 0 || k_host[j] > lim) return fail(PMGRIT_E_ARG, "step index out of range");
  TRY(net_ready(h));
  hipStream_t st = (hipStream_t)hip_stream;
  const InstHost& I = h->inst[inst];
  NetSrc S = h->h_netsrc[inst];
  S.U = U_dev;
  S.Uout = nullptr;
  S.dt = I.lev[level].dt;
  S.kdt = I.prob.kappa * S.dt;
  S.lnc = std::log(S.kdt * (double)I.prob.n_elems * (double)I.prob.n_elems) / 4.0;
  if (level > 0) S.scale = nullptr;  // coarse levels: the step's own dt weights the source
  std::vector<NetPick> pk(nb);
  for (int j = 0; j < nb; ++j) pk[j] = {0, k_host[j]};
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpy(h->d_src_tmp, &S, sizeof(S), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->d_pick_tmp, pk.data(), sizeof(NetPick) * nb, hipMemcpyHostToDevice));
  const int G = S.G;
  HIPCHK(h->net->pack(h->d_src_tmp, h->d_pick_tmp, 0, nb, G, t_dev != nullptr, st));
  const size_t pl = (size_t)nb * G * G;
  HIPCHK(hipMemcpyAsync(x_dev, h->net->x_buf(), sizeof(float) * 3 * pl, hipMemcpyDeviceToDevice, st));
  if (t_dev) HIPCHK(hipMemcpyAsync(t_dev, h->net->t_buf(), sizeof(float) * pl, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(s_dev, h->net->s_buf(), sizeof(double) * nb, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return PMGRIT_OK;
}

// counter-based hash (splitmix64 finaliser) for shuffling
static uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

pmgrit_status pmgrit_net_train(pmgrit_handle* h, const pmgrit_train_opts* opts, const double* const* U_dev,
                               void* hip_stream, pmgrit_train_stats* stats) {
  if (!h || !opts || !U_dev || opts->epochs < 0 || opts->batch < 1 || !(opts->lr >= 0.f))
    return fail(PMGRIT_E_ARG, "bad training arguments");
  TRY(net_ready(h));
  if (!h->net->loaded) return fail(PMGRIT_E_STATE, "no network loaded");
  for (int i = 0; i < h->ninst; ++i)
    if (!U_dev[i]) return fail(PMGRIT_E_ARG, "U_dev[i] is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  auto t0 = std::chrono::steady_clock::now();
  // samples grouped by grid size (a batch has one grid size); batches of the groups interleaved
  std::vector<int> gsz;
  std::vector<std::vector<int>> ginst;
  for (int i = 0; i < h->ninst; ++i) {
    const int G = h->inst[i].Nin + 2;
    size_t q = std::find(gsz.begin(), gsz.end(), G) - gsz.begin();
    if (q == gsz.size()) {
      gsz.push_back(G);
      ginst.emplace_back();
    }
    ginst[q].push_back(i);
  }
  std::vector<NetSrc> src(h->h_netsrc, h->h_netsrc + h->ninst);
  for (int i = 0; i < h->ninst; ++i) src[i].U = U_dev[i];
  NetSrc* d_src = nullptr;
  NetPick* d_pick = nullptr;
  const int64_t total = (int64_t)h->ninst * h->Nt;
  HIPCHK(hipMalloc(&d_src, sizeof(NetSrc) * h->ninst));
  std::unique_ptr<void, void (*)(void*)> g1(d_src, [](void* p) { (void)hipFree(p); });
  HIPCHK(hipMalloc(&d_pick, sizeof(NetPick) * total));
  std::unique_ptr<void, void (*)(void*)> g2(d_pick, [](void* p) { (void)hipFree(p); });
  HIPCHK(hipMemcpy(d_src, src.data(), sizeof(NetSrc) * h->ninst, hipMemcpyHostToDevice));
  for (int G : gsz) HIPCHK(h->net->reserve(opts->batch, G));
  pmgrit_train_stats S;
  std::memset(&S, 0, sizeof(S));
  std::vector<NetPick> order(total);
  for (int ep = 0; ep < opts->epochs; ++ep) {
    // per group: its samples sorted by a counter-based hash of (seed, epoch, sample)
    std::vector<int64_t> gbeg(gsz.size() + 1, 0);
    int64_t o = 0;
    for (size_t q = 0; q < gsz.size(); ++q) {
      std::vector<std::pair<uint64_t, NetPick>> key;
      for (int i : ginst[q])
        for (int k = 0; k < h->Nt; ++k) {
          const uint64_t id = (uint64_t)i * (uint64_t)h->Nt + (uint64_t)k;
          key.push_back({mix64(((uint64_t)opts->seed << 40) ^ ((uint64_t)ep << 32) ^ id), NetPick{i, k}});
        }
      std::sort(key.begin(), key.end(),
                [](const std::pair<uint64_t, NetPick>& a, const std::pair<uint64_t, NetPick>& b) {
                  return a.first < b.first;
                });
      gbeg[q] = o;
      for (auto& kv : key) order[o++] = kv.second;
    }
    gbeg[gsz.size()] = o;
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(d_pick, order.data(), sizeof(NetPick) * total, hipMemcpyHostToDevice));
    double lsum = 0.0;
    int64_t nbat = 0;
    std::vector<int64_t> pos(gbeg.begin(), gbeg.end() - 1);
    for (bool any = true; any;) {
      any = false;
      for (size_t q = 0; q < gsz.size(); ++q) {
        if (pos[q] >= gbeg[q + 1]) continue;
        any = true;
        const int nb = (int)std::min<int64_t>(opts->batch, gbeg[q + 1] - pos[q]);
        HIPCHK(h->net->train_packed(d_src, d_pick + pos[q], nb, gsz[q], opts->lr, st));
        pos[q] += nb;
        double l = 0.0;
        HIPCHK(h->net->read_loss(&l, st));
        if (S.adam_steps == 0) S.loss_first = l;
        ++S.adam_steps;
        lsum += l;
        ++nbat;
      }
    }
    S.loss_last = nbat ? lsum / nbat : 0.0;
    S.epochs_done = ep + 1;
  }
  HIPCHK(hipStreamSynchronize(st));
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = S;
  return PMGRIT_OK;
}

}  // extern "C"
