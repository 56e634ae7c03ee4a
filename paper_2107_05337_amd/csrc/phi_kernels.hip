// phi_kernels.hip -- gfx950 kernels of the spatial solves and the MGRIT point updates.
//
// One workgroup (256 threads, four 64-wide wavefronts) owns one right-hand side and runs the
// whole spatial solve Phi of Sec. 4 for it: right-hand side M u_k + dt f_{k+1}, FP64 residual,
// p-multigrid V-cycles (ILUT smoothing by blocked level-scheduled triangular solves, restriction
// to p = 1, exact p = 1 solve, prolongation) until ||b - A x|| <= tol ||b||, and the MGRIT
// output (next point, or C-point residual).  A chain of consecutive time steps (the F-points of
// one coarse interval) runs inside the same workgroup without leaving the kernel, so a whole
// F-relaxation sweep over every interval of every instance is one launch.
//
// Vectors a step gathers from (triangular-solve work vector y, V-cycle iterate d, FP64 iterate
// x, V-cycle residual s, p = 1 vectors) live in LDS when they fit (template MASK), else in a
// per-workgroup slice of global scratch.  Matrices are read from L2 / MALL.
#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace pmg {

enum : int { kY = 1, kD = 2, kX = 4, kS = 8, kC = 16 };

// offsets of the LDS regions, filled by the host per launch configuration
struct LdsPlan {
  int off_y, off_d, off_x, off_s, off_c, off_sbuf;
  int nmax, n1max;
};

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
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

// out_i = alpha * (A x)_i + beta * z_i   (z may be null), G lanes per row
template <int G, typename AT, typename MV, typename XV, typename ZV, typename OV>
__device__ __forceinline__ void spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                     const MV* __restrict__ v, const XV* x, AT alpha, const ZV* z, AT beta, OV* out) {
  const int g = threadIdx.x & (G - 1);
  for (int i = threadIdx.x / G; i < n; i += kThreads / G) {
    const int k0 = rp[i], k1 = rp[i + 1];
    AT s = 0;
    for (int k = k0 + g; k < k1; k += G) s += (AT)v[k] * (AT)x[ci[k]];
    s = group_sum<G>(s);
    if (g == 0) {
      AT t = alpha * s;
      if (z) t += beta * (AT)z[i];
      out[i] = (OV)t;
    }
  }
}

// FP64 residual r = b - A x, stored in the V-cycle precision; returns this thread's share of ||r||^2
template <int G, typename VT, typename XV>
__device__ __forceinline__ double residual64(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                             const double* __restrict__ A, const XV* x, const double* b, VT* r) {
  const int g = threadIdx.x & (G - 1);
  double part = 0.0;
  for (int i = threadIdx.x / G; i < n; i += kThreads / G) {
    const int k0 = rp[i], k1 = rp[i + 1];
    double s = 0.0;
    for (int k = k0 + g; k < k1; k += G) s += A[k] * (double)x[ci[k]];
    s = group_sum<G>(s);
    if (g == 0) {
      double t = b[i] - s;
      r[i] = (VT)t;
      part += t * t;
    }
  }
  return part;
}

// Blocked level-scheduled triangular solve T out = in (T = L with unit diagonal, or U).
// Per level: phase A forms s_q = in_i - sum_{off-block j} T_ij out_j for every row of the level
// (G lanes per row, shuffle reduction); phase B multiplies each block's s by its dense
// diagonal-block inverse.  With one-row blocks phase B is a scaling and is fused into A.
// `in` may alias `out`.
template <int GA, int GB, typename VT>
__device__ void trsv(const TriDev& T, const VT* in, VT* out, VT* sbuf) {
  const VT* __restrict__ ov = (const VT*)T.ov;
  const VT* __restrict__ dv = (const VT*)T.dval;
  const int* __restrict__ row = T.row;
  const int* __restrict__ orp = T.orp;
  const int* __restrict__ oci = T.oci;
  const int ga = threadIdx.x & (GA - 1);
  if (T.bs == 1) {
    for (int l = 0; l < T.nlev; ++l) {
      const int q0 = T.lev_ptr[l], q1 = T.lev_ptr[l + 1];
      for (int q = q0 + threadIdx.x / GA; q < q1; q += kThreads / GA) {
        const int i = row[q];
        VT s = 0;
        for (int k = orp[q] + ga; k < orp[q + 1]; k += GA) s += ov[k] * out[oci[k]];
        s = group_sum<GA>(s);
        if (ga == 0) out[i] = (in[i] - s) * dv[T.doff[q]];
      }
      __syncthreads();
    }
    return;
  }
  const int gb = threadIdx.x & (GB - 1);
  for (int l = 0; l < T.nlev; ++l) {
    const int q0 = T.lev_ptr[l], q1 = T.lev_ptr[l + 1];
    for (int q = q0 + threadIdx.x / GA; q < q1; q += kThreads / GA) {
      const int i = row[q];
      VT s = 0;
      for (int k = orp[q] + ga; k < orp[q + 1]; k += GA) s += ov[k] * out[oci[k]];
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
      if (gb == 0) out[row[q]] = s;
    }
    __syncthreads();
  }
}

// exact p = 1 solve by fast diagonalisation: c = V diag-solve(V^T c) with one symmetric
// tridiagonal system per mode of the second direction (Thomas, precomputed LDL^T)
__device__ void coarse_solve(const InstDev& I, const LevelDev& L, double* c1, double* c2) {
  const int n1 = I.n1, nn = I.ndof1;
  const double* __restrict__ V = I.V;
  for (int o = threadIdx.x; o < nn; o += kThreads) {
    const int k = o / n1, ix = o - k * n1;
    double s = 0.0;
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
    for (int k = 0; k < n1; ++k) s += Vr[k] * c2[k * n1 + ix];
    c1[o] = s;
  }
  __syncthreads();
}

// one p-multigrid V-cycle from the zero guess on A d = r (Sec. 4, steps 1-5, written in
// correction form: the outer FP64 loop supplies r = b - A x and adds d to x)
template <typename VT>
__device__ void vcycle(const InstDev& I, const LevelDev& L, int nu1, int nu2, const VT* r, VT* d, VT* y, VT* s,
                       double* c1, double* c2, VT* sbuf) {
  const int n = I.ndof;
  const VT* A = (const VT*)L.Avt;
  // step 1: pre-smoothing d = S r, then nu1 - 1 further steps d += S (r - A d)
  trsv<4, 8, VT>(L.L, r, y, sbuf);
  trsv<4, 8, VT>(L.U, y, d, sbuf);
  for (int m = 1; m < nu1; ++m) {
    spmv<8, VT>(n, I.rp, I.ci, A, d, (VT)-1, r, (VT)1, s);
    __syncthreads();
    trsv<4, 8, VT>(L.L, s, y, sbuf);
    trsv<4, 8, VT>(L.U, y, y, sbuf);
    for (int i = threadIdx.x; i < n; i += kThreads) d[i] += y[i];
    __syncthreads();
  }
  // step 2: residual restricted to p = 1, r1 = (M1^L)^{-1} P^T (r - A d)
  spmv<8, VT>(n, I.rp, I.ci, A, d, (VT)-1, r, (VT)1, s);
  __syncthreads();
  spmv<8, VT>(I.ndof1, I.Rrp, I.Rci, (const VT*)I.Rv, s, (VT)1, (const VT*)nullptr, (VT)0, c1);
  __syncthreads();
  // step 3: exact p = 1 solve (FP64)
  coarse_solve(I, L, c1, c2);
  // step 4: prolongation and update d += (Mp^L)^{-1} P e1
  spmv<8, VT>(n, I.Qrp, I.Qci, (const VT*)I.Qv, c1, (VT)1, d, (VT)1, d);
  __syncthreads();
  // step 5: nu2 post-smoothing steps d += S (r - A d)
  for (int m = 0; m < nu2; ++m) {
    spmv<8, VT>(n, I.rp, I.ci, A, d, (VT)-1, r, (VT)1, s);
    __syncthreads();
    trsv<4, 8, VT>(L.L, s, y, sbuf);
    trsv<4, 8, VT>(L.U, y, y, sbuf);
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
  VT* y = (MASK & kY) ? (VT*)(smem + plan.off_y) : (VT*)(ws + 3 * nm);
  VT* d = (MASK & kD) ? (VT*)(smem + plan.off_d) : (VT*)(ws + 4 * nm);
  VT* s = (MASK & kS) ? (VT*)(smem + plan.off_s) : (VT*)(ws + 5 * nm);
  double* c1 = (MASK & kC) ? (double*)(smem + plan.off_c) : ws + 6 * nm;
  double* c2 = c1 + plan.n1max;

  double* Vl = P.vtab ? P.vtab[job.inst * kMaxLevels + job.level] : nullptr;
  const double* Gl = (P.gtab && job.level > 0) ? P.gtab[job.inst * kMaxLevels + job.level] : nullptr;
  const double stol2 = P.stol * P.stol;
  int total = 0;
  for (int st = 0; st < job.len; ++st) {
    const int k = job.k0 + st;  // step from point k to point k + 1
    const double* g1 = Gl ? Gl + (int64_t)(k + 1) * n : nullptr;
    double* tgt = Vl ? Vl + (int64_t)(k + 1) * n : nullptr;
    // right-hand side and initial iterate
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
      spmv<8, double>(n, I.rp, I.ci, I.M, vk, 1.0, job.level == 0 ? I.F : (const double*)nullptr, c, b);
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
      part = residual64<8, VT>(n, I.rp, I.ci, L.A64, x, b, r);
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
      vcycle<VT>(I, L, P.nu1, P.nu2, r, d, y, s, c1, c2, sbuf);
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
  __shared__ double red[kThreads / 64];
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
    case 31: return phi_kernel<VT, 31>;
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

hipError_t phi_launch(int fp32, int mask, int lds_bytes, const PhiParams& P, const int* plan6, int nmax, int n1max,
                      int nblocks, hipStream_t st) {
  LdsPlan plan{plan6[0], plan6[1], plan6[2], plan6[3], plan6[4], plan6[5], nmax, n1max};
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
  hipLaunchKernelGGL(norm_reduce_kernel, dim3(ninst), dim3(kThreads), 0, st, nrm2, begin, out);
  return hipGetLastError();
}

}  // namespace pmg
