// phi_kernels.hip -- gfx950 kernels of the spatial solves and the MGRIT point updates.
//
// One workgroup (1024 threads, sixteen 64-wide wavefronts) owns one right-hand side and runs the
// whole spatial solve Phi of Sec. 4 for it: right-hand side M u_k + dt f_{k+1}, FP64 residual,
// p-multigrid V-cycles (ILUT smoothing, restriction to p = 1, exact p = 1 solve, prolongation)
// until ||b - A x|| <= tol ||b||, and the MGRIT output (next point, or C-point residual).  A
// chain of consecutive time steps (the F-points of one coarse interval) runs inside the same
// workgroup, so a whole F-relaxation sweep over every interval of every instance is one launch.
//
// Operators: A_l, M and both transfers are sums of Kronecker products of banded 1D matrices on
// the separable single-patch geometries, so they are applied by sum factorisation from small
// band arrays (no sparse-matrix streaming).  The ILUT factors are general sparse: they are
// applied by blocked level-scheduled triangular solves whose next level is prefetched into
// registers while the current one computes; the workgroup then synchronises on LDS only.
// Work vectors live in LDS when they fit (template MASK), else in a per-workgroup slice of
// global scratch.
#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace pmg {

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// barrier that orders LDS traffic only (global loads in flight stay in flight)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// sum over the workgroup, result on every thread (deterministic order)
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = group_sum<64>(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) s += red[i];
  return s;
}

template <typename T>
__device__ __forceinline__ const T* band_ptr(const BandDev& B);
template <>
__device__ __forceinline__ const double* band_ptr<double>(const BandDev& B) {
  return B.f64;
}
template <>
__device__ __forceinline__ const float* band_ptr<float>(const BandDev& B) {
  return (const float*)B.vt;
}

// ---------------------------------------------------------------------------------------
// sum-factorised Kronecker passes
// ---------------------------------------------------------------------------------------

// first-direction pass: T[r][o] = sum_d B[o][d] * in[r][o + lo + d] for r < nrows, o < B.rows
// (in has nin columns; band entries outside the input range are zero, their index is clamped)
template <typename AT, typename IT, typename OT>
__device__ __forceinline__ void pass_x(int nrows, int nin, const BandDev& Bd, const IT* in, OT* out) {
  const AT* __restrict__ B = band_ptr<AT>(Bd);
  const int nout = Bd.rows, w = Bd.w, lo = Bd.lo;
  const int tot = nrows * nout;
  for (int t = threadIdx.x; t < tot; t += kThreads) {
    const int r = t / nout, o = t - r * nout;
    const IT* src = in + r * nin;
    const AT* b = B + o * w;
    AT s = 0;
    for (int d = 0; d < w; ++d) {
      int j = o + lo + d;
      j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
      s += b[d] * (AT)src[j];
    }
    out[t] = (OT)s;
  }
}

// second-direction pass: out[o][c] = alpha * sc(o,c) * sum_d B[o][d] * T[o + lo + d][c]
//                                    + beta * z[o][c] (+ out[o][c] if acc)
// for o < B.rows, c < ncols; T has nin rows.  sc(o,c) = scy[o] * scx[c] when scy is given.
// Returns this thread's share of sum out^2 (used for residual norms).
template <typename AT, typename TT, typename ZT, typename OT>
__device__ __forceinline__ double pass_y(int ncols, int nin, const BandDev& Bd, const TT* T, AT alpha, const ZT* z,
                                         AT beta, bool acc, const double* scy, const double* scx, OT* out) {
  const AT* __restrict__ B = band_ptr<AT>(Bd);
  const int nout = Bd.rows, w = Bd.w, lo = Bd.lo;
  const int tot = nout * ncols;
  double part = 0.0;
  for (int t = threadIdx.x; t < tot; t += kThreads) {
    const int o = t / ncols, c = t - o * ncols;
    const AT* b = B + o * w;
    AT s = 0;
    for (int d = 0; d < w; ++d) {
      int j = o + lo + d;
      j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
      s += b[d] * (AT)T[j * ncols + c];
    }
    AT v = alpha * s;
    if (scy) v *= (AT)(scy[o] * scx[c]);
    if (z) v += beta * (AT)z[t];
    if (acc) v += (AT)out[t];
    out[t] = (OT)v;
    part += (double)v * (double)v;
  }
  return part;
}

// out = beta z - A_l x with A_l = My (x) X1 + c Ky (x) Mx2 (temp: nin x nin scratch, may not
// alias x or out).  Returns this thread's share of ||out||^2.
template <typename AT, typename XT, typename ZT, typename OT, typename TT>
__device__ double apply_A(const InstDev& I, const LevelDev& L, const XT* x, const ZT* z, OT* out, TT* tmp) {
  const int n = I.nin;
  pass_x<AT>(n, n, L.X1, x, tmp);
  __syncthreads();
  pass_y<AT>(n, n, I.My, tmp, (AT)-1, z, (AT)1, false, nullptr, nullptr, out);
  __syncthreads();
  pass_x<AT>(n, n, I.Mx2, x, tmp);
  __syncthreads();
  double part = pass_y<AT>(n, n, I.Ky, tmp, (AT)(-L.c), (const ZT*)nullptr, (AT)0, true, nullptr, nullptr, out);
  __syncthreads();
  return part;
}

// ---------------------------------------------------------------------------------------
// blocked level-scheduled triangular solves
// ---------------------------------------------------------------------------------------

// Prefetched path: T y = in (T = L with unit diagonal, or U), solution written to y (which may
// alias in).  Thread (r, g) = (row slot tid / 8, lane tid % 8).  Per level: phase A forms
// s_r = in_i - sum_{off-block j} T_ij y_j (its entries were loaded during the previous level),
// phase B multiplies each block's s by its dense diagonal-block inverse (loaded at the start of
// the level, while phase A runs).  y and sbuf are in LDS, so the barriers fence LDS only.
template <typename VT>
__device__ void trsv_fast(const TriDev& T, const VT* in, VT* y, VT* sbuf) {
  const VT* __restrict__ ov = (const VT*)T.ov;
  const VT* __restrict__ dv = (const VT*)T.dval;
  const int r = threadIdx.x / kTG, g = threadIdx.x & (kTG - 1);
  int q0 = T.lev_ptr[0], q1 = T.lev_ptr[1];
  int row = -1, na = 0;  // na: valid entries of this lane (padding never touches y: stale LDS
                         // words of another type may hold NaN patterns)
  VT av[kTMA];
  int ac[kTMA];
  {
    const int q = q0 + r;
    int k0 = 0, k1 = 0;
    if (q < q1) {
      row = T.row[q];
      k0 = T.orp[q];
      k1 = T.orp[q + 1];
    }
    na = k1 - k0;
#pragma unroll
    for (int j = 0; j < kTMA; ++j) {
      const int k = k0 + g + j * kTG;
      av[j] = k < k1 ? ov[k] : (VT)0;
      ac[j] = k < k1 ? T.oci[k] : 0;
    }
  }
  for (int l = 0; l < T.nlev; ++l) {
    // dense row of this level's block (consumed after phase A)
    VT bv[kTMB];
    int bq0 = 0, bcnt = 0;
    {
      const int q = q0 + r;
      int64_t off = 0;
      if (q < q1) {
        bq0 = T.dq0[q];
        bcnt = T.dcnt[q];
        off = T.doff[q];
      }
#pragma unroll
      for (int j = 0; j < kTMB; ++j) {
        const int c = g + j * kTG;
        bv[j] = c < bcnt ? dv[off + c] : (VT)0;
      }
    }
    // prefetch the off-block entries of the next level
    const int nq0 = q1, nq1 = l + 1 < T.nlev ? T.lev_ptr[l + 2] : q1;
    int nrow = -1, nna = 0;
    VT nv[kTMA];
    int nc[kTMA];
    {
      const int q = nq0 + r;
      int k0 = 0, k1 = 0;
      if (q < nq1) {
        nrow = T.row[q];
        k0 = T.orp[q];
        k1 = T.orp[q + 1];
      }
      nna = k1 - k0;
#pragma unroll
      for (int j = 0; j < kTMA; ++j) {
        const int k = k0 + g + j * kTG;
        nv[j] = k < k1 ? ov[k] : (VT)0;
        nc[j] = k < k1 ? T.oci[k] : 0;
      }
    }
    // phase A
    VT s = 0;
#pragma unroll
    for (int j = 0; j < kTMA; ++j) {
      const VT yv = y[ac[j]];
      s += (g + j * kTG < na) ? av[j] * yv : (VT)0;
    }
    s = group_sum<kTG>(s);
    if (g == 0 && row >= 0) sbuf[r] = in[row] - s;
    lds_barrier();
    // phase B
    s = 0;
#pragma unroll
    for (int j = 0; j < kTMB; ++j) {
      const int c = g + j * kTG;
      const VT sv = sbuf[bq0 + (c < bcnt ? c : 0)];
      s += (c < bcnt) ? bv[j] * sv : (VT)0;
    }
    s = group_sum<kTG>(s);
    if (g == 0 && row >= 0) y[row] = s;
    lds_barrier();
    q0 = nq0;
    q1 = nq1;
    row = nrow;
    na = nna;
#pragma unroll
    for (int j = 0; j < kTMA; ++j) {
      av[j] = nv[j];
      ac[j] = nc[j];
    }
  }
}

// General path (any schedule, y in LDS or global): same two phases with loops, full barriers.
template <typename VT>
__device__ void trsv_general(const TriDev& T, const VT* in, VT* y, VT* sbuf) {
  constexpr int GA = 8, GB = 8;
  const VT* __restrict__ ov = (const VT*)T.ov;
  const VT* __restrict__ dv = (const VT*)T.dval;
  const int ga = threadIdx.x & (GA - 1), gb = threadIdx.x & (GB - 1);
  for (int l = 0; l < T.nlev; ++l) {
    const int q0 = T.lev_ptr[l], q1 = T.lev_ptr[l + 1];
    for (int q = q0 + threadIdx.x / GA; q < q1; q += kThreads / GA) {
      const int i = T.row[q];
      VT s = 0;
      for (int k = T.orp[q] + ga; k < T.orp[q + 1]; k += GA) s += ov[k] * y[T.oci[k]];
      s = group_sum<GA>(s);
      if (ga == 0) sbuf[q - q0] = in[i] - s;
    }
    __syncthreads();
    for (int q = q0 + threadIdx.x / GB; q < q1; q += kThreads / GB) {
      const int c0 = T.dq0[q], cn = T.dcnt[q];
      const VT* __restrict__ dr = dv + T.doff[q];
      VT s = 0;
      for (int c = gb; c < cn; c += GB) s += dr[c] * sbuf[c0 + c];
      s = group_sum<GB>(s);
      if (gb == 0) y[T.row[q]] = s;
    }
    __syncthreads();
  }
}

template <typename VT, bool YLDS>
__device__ __forceinline__ void trsv(const TriDev& T, const VT* in, VT* y, VT* sbuf) {
  if (YLDS && T.fast)
    trsv_fast<VT>(T, in, y, sbuf);
  else
    trsv_general<VT>(T, in, y, sbuf);
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// exact p = 1 solve: fast diagonalisation c = V diag-solve(V^T c), one symmetric tridiagonal
// system per mode of the second direction (Thomas, precomputed LDL^T).  c1 in / out, c2 temp.
// ---------------------------------------------------------------------------------------
__device__ void coarse_solve(const InstDev& I, const LevelDev& L, double* c1, double* c2) {
  const int n1 = I.n1, nn = I.ndof1;
  const double* __restrict__ V = I.V;
  for (int o = threadIdx.x; o < nn; o += kThreads) {
    const int k = o / n1, ix = o - k * n1;
    double s = 0.0;
#pragma unroll 8
    for (int iy = 0; iy < n1; ++iy) s += V[iy * n1 + k] * c1[iy * n1 + ix];
    c2[o] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n1; k += kThreads) {
    double* rw = c2 + k * n1;
    const double* __restrict__ tl = L.tl + k * n1;
    const double* __restrict__ td = L.tdinv + k * n1;
    double yp = rw[0];
    rw[0] = yp * td[0];
    for (int i = 1; i < n1; ++i) {
      double yv = rw[i] - tl[i] * yp;
      rw[i] = yv * td[i];
      yp = yv;
    }
    double xn = rw[n1 - 1];
    for (int i = n1 - 2; i >= 0; --i) {
      xn = rw[i] - tl[i + 1] * xn;
      rw[i] = xn;
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < nn; o += kThreads) {
    const int iy = o / n1, ix = o - iy * n1;
    double s = 0.0;
    const double* __restrict__ Vr = V + iy * n1;
#pragma unroll 8
    for (int k = 0; k < n1; ++k) s += Vr[k] * c2[k * n1 + ix];
    c1[o] = s;
  }
  __syncthreads();
}

// one p-multigrid V-cycle from the zero guess on A d = r (Sec. 4, steps 1-5, in correction
// form: the outer FP64 loop supplies r = b - A x and adds d to x).
// Buffers: y (nin^2 doubles, LDS first), s (>= max(nin^2 VT, n1^2 doubles)), d (nin^2 VT).
template <typename VT, int MASK>
__device__ void vcycle(const InstDev& I, const LevelDev& L, int nu1, int nu2, const VT* r, VT* d, VT* y, VT* s,
                       VT* sbuf) {
  constexpr bool YL = MASK & kY;
  const int n = I.ndof;
  // step 1: pre-smoothing d = S r, then nu1 - 1 further steps d += S (r - A d)
  trsv<VT, YL>(L.L, r, y, sbuf);
  trsv<VT, YL>(L.U, y, y, sbuf);
  for (int i = threadIdx.x; i < n; i += kThreads) d[i] = y[i];
  __syncthreads();
  for (int m = 1; m < nu1; ++m) {
    apply_A<VT>(I, L, d, r, s, y);
    trsv<VT, YL>(L.L, s, y, sbuf);
    trsv<VT, YL>(L.U, y, y, sbuf);
    for (int i = threadIdx.x; i < n; i += kThreads) d[i] += y[i];
    __syncthreads();
  }
  // step 2: residual restricted to p = 1, r1 = (M1^L)^{-1} P^T (r - A d); r1 lands in s
  apply_A<VT>(I, L, d, r, s, y);
  double* c1 = (double*)s;
  double* c2 = (double*)y;
  pass_x<VT>(I.nin, I.nin, I.PxT, s, y);  // nin rows x n1 columns
  __syncthreads();
  pass_y<VT>(I.n1, I.nin, I.PyT, y, (VT)1, (const VT*)nullptr, (VT)0, false, I.il1_y, I.il1_x, c1);
  __syncthreads();
  // step 3: exact p = 1 solve (FP64)
  coarse_solve(I, L, c1, c2);
  // step 4: prolongation and update d += (Mp^L)^{-1} P e1
  pass_x<VT>(I.n1, I.n1, I.Px, c1, y);  // n1 rows x nin columns
  __syncthreads();
  pass_y<VT>(I.nin, I.n1, I.Py, y, (VT)1, (const VT*)nullptr, (VT)0, true, I.ilp_y, I.ilp_x, d);
  __syncthreads();
  // step 5: nu2 post-smoothing steps d += S (r - A d)
  for (int m = 0; m < nu2; ++m) {
    apply_A<VT>(I, L, d, r, s, y);
    trsv<VT, YL>(L.L, s, y, sbuf);
    trsv<VT, YL>(L.U, y, y, sbuf);
    for (int i = threadIdx.x; i < n; i += kThreads) d[i] += y[i];
    __syncthreads();
  }
}

template <typename VT, int MASK>
__global__ void __launch_bounds__(kThreads) phi_kernel(PhiParams P, LdsPlan plan) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PhiJob job = P.jobs[blockIdx.x];
  const InstDev& I = P.inst[job.inst];
  const LevelDev& L = I.lev[job.level];
  const int n = I.ndof;
  double* red = (double*)smem;
  VT* sbuf = (VT*)(smem + plan.off_sbuf);
  double* ws = P.ws + (int64_t)blockIdx.x * P.ws_stride;
  const int nm = plan.nmax;
  double* b = ws;
  VT* r = (VT*)(ws + nm);
  double* x = (MASK & kX) ? (double*)(smem + plan.off_x) : ws + 2 * nm;
  double* yd = (MASK & kY) ? (double*)(smem + plan.off_y) : ws + 3 * nm;  // FP64-sized slot
  VT* y = (VT*)yd;
  VT* d = (MASK & kD) ? (VT*)(smem + plan.off_d) : (VT*)(ws + 4 * nm);
  VT* s = (MASK & kS) ? (VT*)(smem + plan.off_s) : (VT*)(ws + 5 * nm);

  double* Vl = P.vtab ? P.vtab[job.inst * kMaxLevels + job.level] : nullptr;
  const double* Gl = (P.gtab && job.level > 0) ? P.gtab[job.inst * kMaxLevels + job.level] : nullptr;
  const double stol2 = P.stol * P.stol;
  int total = 0;
  for (int st = 0; st < job.len; ++st) {
    const int k = job.k0 + st;  // step from point k to point k + 1
    const double* g1 = Gl ? Gl + (int64_t)(k + 1) * n : nullptr;
    double* tgt = Vl ? Vl + (int64_t)(k + 1) * n : nullptr;
    // right-hand side b = M v_k + dt f_{k+1} (level 0) or M v_k, and the initial iterate
    if (P.mode == kModeGiven) {
      const double* bg = P.bgiven + (int64_t)blockIdx.x * n;
      const double* xg = P.xgiven + (int64_t)blockIdx.x * n;
      for (int i = threadIdx.x; i < n; i += kThreads) {
        b[i] = bg[i];
        x[i] = xg[i];
      }
    } else {
      const double* vk = Vl + (int64_t)k * n;
      const double c = job.level == 0 ? I.scale[k + 1] : 0.0;
      pass_x<double>(I.nin, I.nin, I.Mx, vk, yd);
      __syncthreads();
      pass_y<double>(I.nin, I.nin, I.My, yd, 1.0, job.level == 0 ? I.F : (const double*)nullptr, c, false,
                     nullptr, nullptr, b);
      // initial iterate: 0 zero; 1 previous point; 2 current target at level 0 (the previous
      // MGRIT iterate), previous point at coarse levels (their state restarts from zero)
      const bool prev = P.guess == 1 || (P.guess == 2 && job.level > 0);
      for (int i = threadIdx.x; i < n; i += kThreads) x[i] = prev ? vk[i] : (P.guess == 2 ? tgt[i] : 0.0);
    }
    __syncthreads();
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) part += b[i] * b[i];
    const double bn2 = block_sum(part, red);
    int cyc = 0;
    if (bn2 == 0.0) {  // zero right-hand side: the solution is exactly zero
      for (int i = threadIdx.x; i < n; i += kThreads) x[i] = 0.0;
      __syncthreads();
    }
    for (; bn2 != 0.0;) {
      // FP64 residual r = b - A x (stored in the V-cycle precision) and its norm
      part = 0.0;
      if constexpr (sizeof(VT) == 8) {
        part = apply_A<double>(I, L, x, b, r, yd);
      } else {
        // residual in FP64 through the FP64 temp, then rounded into r
        double* rr = (double*)(ws + 5 * nm);  // FP64 residual staging in global scratch
        part = apply_A<double>(I, L, x, b, rr, yd);
        for (int i = threadIdx.x; i < n; i += kThreads) r[i] = (VT)rr[i];
      }
      const double rn2 = block_sum(part, red);
      if (!(rn2 <= 1.0e300)) {  // NaN or Inf
        if (threadIdx.x == 0) atomicOr(P.status, 1);
        break;
      }
      if (rn2 <= stol2 * bn2) break;
      if (cyc >= P.maxcyc) {
        if (threadIdx.x == 0) atomicOr(P.status, 2);
        break;
      }
      vcycle<VT, MASK>(I, L, P.nu1, P.nu2, r, d, y, s, sbuf);
      for (int i = threadIdx.x; i < n; i += kThreads) x[i] += (double)d[i];
      __syncthreads();
      ++cyc;
    }
    total += cyc;
    // output
    if (P.mode == kModeChain) {
      for (int i = threadIdx.x; i < n; i += kThreads) tgt[i] = x[i] + (g1 ? g1[i] : 0.0);
    } else if (P.mode == kModeResidual) {
      double* ro = P.gtab[job.inst * kMaxLevels + job.level + 1] + (int64_t)job.outj * n;
      part = 0.0;
      for (int i = threadIdx.x; i < n; i += kThreads) {
        double v = x[i] + (g1 ? g1[i] : 0.0) - tgt[i];
        ro[i] = v;
        part += v * v;
      }
      const double r2 = block_sum(part, red);
      if (threadIdx.x == 0) P.nrm2[blockIdx.x] = r2;
    } else {
      double* xg = P.xgiven + (int64_t)blockIdx.x * n;
      for (int i = threadIdx.x; i < n; i += kThreads) xg[i] = x[i];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    P.vcount[blockIdx.x] += total;
    if (P.vlast) P.vlast[blockIdx.x] = total;
  }
}

// ------------------------------------------------------------------------------------------
// small MGRIT kernels
// ------------------------------------------------------------------------------------------

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void copy_kernel(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// coarse-grid correction of the C-points: V_l[j m] += V_{l+1}[j], j = 1 .. ncoarse
__global__ void correct_kernel(double* __restrict__ Vl, const double* __restrict__ Vc, int ndof, int m,
                               int ncoarse) {
  const int64_t tot = (int64_t)ncoarse * ndof;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / ndof + 1, i = t - (j - 1) * ndof;
    Vl[j * m * (int64_t)ndof + i] += Vc[j * (int64_t)ndof + i];
  }
}

// per instance: sum of the residual norms of its workgroups [begin[i], begin[i+1])
__global__ void norm_reduce_kernel(const double* __restrict__ nrm2, const int* __restrict__ begin,
                                   double* __restrict__ out) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = begin[i] + threadIdx.x; j < begin[i + 1]; j += blockDim.x) s += nrm2[j];
  s = group_sum<64>(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += red[w];
    out[i] = t;
  }
}

// ------------------------------------------------------------------------------------------
// host-side launch helpers (called from the driver)
// ------------------------------------------------------------------------------------------

using PhiFn = void (*)(PhiParams, LdsPlan);

template <typename VT>
static PhiFn pick(int mask) {
  switch (mask) {
    case 15: return phi_kernel<VT, 15>;
    case 7: return phi_kernel<VT, 7>;
    case 3: return phi_kernel<VT, 3>;
    case 1: return phi_kernel<VT, 1>;
    default: return phi_kernel<VT, 0>;
  }
}

hipError_t phi_prepare(int fp32, int mask, int lds_bytes) {
  PhiFn f = fp32 ? pick<float>(mask) : pick<double>(mask);
  return hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t phi_launch(int fp32, int mask, int lds_bytes, const PhiParams& P, const LdsPlan& plan, int nblocks,
                      hipStream_t st) {
  PhiFn f = fp32 ? pick<float>(mask) : pick<double>(mask);
  hipLaunchKernelGGL(f, dim3(nblocks), dim3(kThreads), lds_bytes, st, P, plan);
  return hipGetLastError();
}

hipError_t fill_launch(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t copy_launch(double* dst, const double* src, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t correct_launch(double* Vl, const double* Vc, int ndof, int m, int ncoarse, hipStream_t st) {
  int64_t tot = (int64_t)ncoarse * ndof;
  if (tot <= 0) return hipSuccess;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(correct_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Vl, Vc, ndof, m, ncoarse);
  return hipGetLastError();
}

hipError_t norm_reduce_launch(const double* nrm2, const int* begin, double* out, int ninst, hipStream_t st) {
  hipLaunchKernelGGL(norm_reduce_kernel, dim3(ninst), dim3(256), 0, st, nrm2, begin, out);
  return hipGetLastError();
}

}  // namespace pmg
