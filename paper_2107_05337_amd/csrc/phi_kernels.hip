// phi_kernels.hip -- gfx950 kernels of the spatial solves and the MGRIT point updates.
//
// One workgroup (512 or 1024 threads, see Build) owns one right-hand side and runs the
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
// global scratch; when the triangular-solve vector y is in global memory, the solves read the
// grid lines they couple to from an LDS window.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_types.hpp"

namespace pmg {

// Global-memory pointer type.  Pointers read from descriptors in memory are otherwise generic
// and their loads become flat loads, which also count against the LDS wait counter: every LDS
// wait and LDS-only barrier would then wait for all prefetches in flight.
template <class T>
using G = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ const G<T>* gp(const T* p) {
  return (const G<T>*)p;
}
// LDS pointer type
template <class T>
using L3 = __attribute__((address_space(3))) T;

// Kernel builds: OCC 1 runs 512 threads (4 lanes per triangular-solve row, 128 row slots per
// level, a 256-register budget per thread), OCC 2 the same limited to 128 registers (two
// workgroups per CU), OCC 3 1024 threads (8 lanes per row, 128 registers): shorter per-lane
// work in every phase of one solve.  OCC 4 runs 512 threads with 8 lanes per row (64 row slots
// per level, 256 registers), for schedules of at most 64 rows per level.
template <int OCC>
struct Build {
  static constexpr int NT = OCC == 3 ? 1024 : 512, TG = (OCC == 3 || OCC == 4) ? 8 : 4;
  // wave tile width (16 x 16 blocks) of the p = 1 transforms: narrower where registers are scarce
  static constexpr int GBC = (OCC == 1 || OCC == 4) ? 4 : 1;
};

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
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = group_sum<64>(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

template <typename T>
__device__ __forceinline__ const G<T>* band_ptr(const BandDev& B);
template <>
__device__ __forceinline__ const G<double>* band_ptr<double>(const BandDev& B) {
  return gp(B.f64);
}
template <>
__device__ __forceinline__ const G<float>* band_ptr<float>(const BandDev& B) {
  return gp((const float*)B.vt);
}

// ---------------------------------------------------------------------------------------
// sum-factorised Kronecker passes
// ---------------------------------------------------------------------------------------

constexpr int kBandMax = 11;  // widest 1D band: 2p + 1 at p = 5

// first-direction pass: T[r][o] = sum_d B[o][d] * in[r][o + lo + d] for r < nrows, o < B.rows
// (in has nin columns; band entries outside the input range are zero, their index is clamped).
// Thread (o, g) keeps band row o in registers and covers rows g, g + NT / nout, ...
template <int NT, typename AT, typename IT, typename OT>
__device__ __forceinline__ void pass_x(int nrows, int nin, const BandDev& Bd, const IT* in, OT* out) {
  const G<AT>* __restrict__ B = band_ptr<AT>(Bd);
  const int nout = Bd.rows, w = Bd.w, lo = Bd.lo;
  if (w <= kBandMax && nout <= NT) {
    const int groups = NT / nout;
    const int o = threadIdx.x % nout, g = threadIdx.x / nout;
    if (g >= groups) return;
    AT b[kBandMax];
    int jj[kBandMax];
#pragma unroll
    for (int d = 0; d < kBandMax; ++d) {
      b[d] = d < w ? B[o * w + d] : (AT)0;
      int j = o + lo + d;
      jj[d] = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
    }
    for (int r = g; r < nrows; r += groups) {
      const IT* src = in + r * nin;
      AT s = 0;
#pragma unroll
      for (int d = 0; d < kBandMax; ++d) s += b[d] * (AT)src[jj[d]];
      out[r * nout + o] = (OT)s;
    }
    return;
  }
  const int tot = nrows * nout;
  for (int t = threadIdx.x; t < tot; t += NT) {
    const int r = t / nout, o = t - r * nout;
    const IT* src = in + r * nin;
    const G<AT>* b = B + o * w;
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
template <int NT, typename AT, typename TT, typename ZT, typename OT>
__device__ __forceinline__ double pass_y(int ncols, int nin, const BandDev& Bd, const TT* T, AT alpha, const ZT* z,
                                         AT beta, bool acc, const double* scy, const double* scx, OT* out) {
  const G<AT>* __restrict__ B = band_ptr<AT>(Bd);
  const int nout = Bd.rows, w = Bd.w, lo = Bd.lo;
  const int tot = nout * ncols;
  double part = 0.0;
  for (int t = threadIdx.x; t < tot; t += NT) {
    const int o = t / ncols, c = t - o * ncols;
    const G<AT>* b = B + o * w;
    AT s = 0;
    if (w <= kBandMax) {
      // the row's coefficients first, all in flight together (kept ahead of their use even
      // where registers are scarce)
      AT bb[kBandMax];
#pragma unroll
      for (int d = 0; d < kBandMax; ++d) bb[d] = b[d < w ? d : w - 1];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int d = 0; d < kBandMax; ++d) {
        int j = o + lo + d;
        j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
        s += (d < w ? bb[d] : (AT)0) * (AT)T[j * ncols + c];
      }
    } else {
      for (int d = 0; d < w; ++d) {
        int j = o + lo + d;
        j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
        s += b[d] * (AT)T[j * ncols + c];
      }
    }
    AT v = alpha * s;
    if (scy) v *= (AT)(gp(scy)[o] * gp(scx)[c]);
    if (z) v += beta * (AT)z[t];
    if (acc) v += (AT)out[t];
    out[t] = (OT)v;
    part += (double)v * (double)v;
  }
  return part;
}

// Both first-direction passes of A_l at once (bands of equal shape): t1 = X1 pass, t2 = Mx2 pass
// of the same input, each tap of the input read once for both.
template <int NT, typename AT, typename IT, typename OT>
__device__ __forceinline__ void pass_x2(int nrows, int nin, const BandDev& B1d, const BandDev& B2d, const IT* in,
                                        OT* out1, OT* out2) {
  const G<AT>* __restrict__ B1 = band_ptr<AT>(B1d);
  const G<AT>* __restrict__ B2 = band_ptr<AT>(B2d);
  const int nout = B1d.rows, w = B1d.w, lo = B1d.lo;
  const int groups = NT / nout;
  const int o = threadIdx.x % nout, g = threadIdx.x / nout;
  if (g >= groups) return;
  AT b1[kBandMax], b2[kBandMax];
  int jj[kBandMax];
#pragma unroll
  for (int d = 0; d < kBandMax; ++d) {
    b1[d] = d < w ? B1[o * w + d] : (AT)0;
    b2[d] = d < w ? B2[o * w + d] : (AT)0;
    const int j = o + lo + d;
    jj[d] = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
  }
  for (int r = g; r < nrows; r += groups) {
    const IT* src = in + r * nin;
    AT s1 = 0, s2 = 0;
#pragma unroll
    for (int d = 0; d < kBandMax; ++d) {
      const AT v = (AT)src[jj[d]];
      s1 += b1[d] * v;
      s2 += b2[d] * v;
    }
    out1[r * nout + o] = (OT)s1;
    out2[r * nout + o] = (OT)s2;
  }
}

// Both second-direction passes at once: out = (a1 (B1 pass of T1) + beta z) + a2 (B2 pass of T2),
// bands of equal shape, rounded in the same order as two pass_y calls (the second accumulating),
// so fused and unfused residuals agree bitwise.  Returns this thread's share of sum out^2.
template <int NT, typename AT, typename TT, typename ZT, typename OT>
__device__ __forceinline__ double pass_y2(int ncols, int nin, const BandDev& B1d, const BandDev& B2d, const TT* T1,
                                          const TT* T2, AT a1, AT a2, const ZT* z, AT beta, OT* out) {
  const G<AT>* __restrict__ B1 = band_ptr<AT>(B1d);
  const G<AT>* __restrict__ B2 = band_ptr<AT>(B2d);
  const int nout = B1d.rows, w = B1d.w, lo = B1d.lo;
  const int tot = nout * ncols;
  double part = 0.0;
  for (int t = threadIdx.x; t < tot; t += NT) {
    const int o = t / ncols, c = t - o * ncols;
    const G<AT>* b1 = B1 + o * w;
    const G<AT>* b2 = B2 + o * w;
    AT c1[kBandMax], c2[kBandMax];
#pragma unroll
    for (int d = 0; d < kBandMax; ++d) {
      c1[d] = b1[d < w ? d : w - 1];
      c2[d] = b2[d < w ? d : w - 1];
    }
    __builtin_amdgcn_sched_barrier(0);
    AT s1 = 0, s2 = 0;
#pragma unroll
    for (int d = 0; d < kBandMax; ++d) {
      int j = o + lo + d;
      j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
      s1 += (d < w ? c1[d] : (AT)0) * (AT)T1[j * ncols + c];
      s2 += (d < w ? c2[d] : (AT)0) * (AT)T2[j * ncols + c];
    }
    AT v = a1 * s1;
    if (z) v += beta * (AT)z[t];
    v += a2 * s2;
    out[t] = (OT)v;
    part += (double)v * (double)v;
  }
  return part;
}

// LDS staging of the band passes whose vectors are in global memory (y not in LDS): per chunk of
// rows the band entries and the input rows are copied into LDS by every thread, many loads in
// flight per thread, and the outputs are formed from LDS.  The direct passes pay one global
// load latency per output row and thread in sequence; here a chunk costs a few.  Each output is
// summed in the same order and with the same operations as in the direct passes, so the outputs
// agree bitwise.  p = null, or an area too small for the pass: the direct pass.  Vectors are read
// through generic pointers (any of them may be in LDS).
struct Stg {
  unsigned char* p = nullptr;
  int bytes = 0;
};
constexpr int kStU = 8;
// the builds that stage: y in global memory, the 512-thread build with the full register budget
template <int MASK, int OCC>
struct Staged {
  static constexpr bool value = !(MASK & kY) && OCC == 1;
};

__device__ __forceinline__ int al16(int b) { return (b + 15) / 16 * 16; }

// copies n elements of src into dst (and of src2 into dst2 when given), kCopyU loads of each in
// flight per thread before the first store
constexpr int kCopyU = 16;
template <int NT, typename T, typename S>
__device__ __forceinline__ void stage_copy(L3<T>* dst, const S* src, int n, L3<T>* dst2 = nullptr,
                                           const S* src2 = nullptr) {
  for (int e0 = threadIdx.x; e0 < n; e0 += kCopyU * NT) {
    T v[kCopyU], v2[kCopyU];
#pragma unroll
    for (int u = 0; u < kCopyU; ++u) {
      const int e = e0 + u * NT;
      v[u] = e < n ? (T)src[e] : (T)0;
      if (src2) v2[u] = e < n ? (T)src2[e] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < kCopyU; ++u) {
      const int e = e0 + u * NT;
      if (e < n) {
        dst[e] = v[u];
        if (src2) dst2[e] = v2[u];
      }
    }
  }
}

// first index >= base that this thread owns in a pass over outputs 0, 1, ... (index mod NT)
template <int NT>
__device__ __forceinline__ int own_from(int base) {
  return ((int)threadIdx.x - base % NT + NT) % NT;
}

// Compute of the staged passes with bands of at most kBandMax entries: band rows staged at stride kBS
// with zeros past w, so every output takes kBandMax taps exactly as the direct passes do (same
// products, same order: the values agree bitwise).  Register blocking over four outputs:
// first-direction passes give each thread one output column o of four rows, its band row loaded once;
// second-direction passes give each thread four consecutive output rows of one column, the
// 4 + kBandMax - 1 input values they share loaded once.  The norms' partial sums are grouped by thread
// differently from the direct passes (their roundings may differ in the last place).
constexpr int kBS = kBandMax + 1;

// band rows o0 .. o0 + n - 1 of B (and B2) into dst (dst2) at stride kBS, zero past w
template <int NT, typename AT>
__device__ __forceinline__ void stage_band(L3<AT>* dst, const G<AT>* __restrict__ B, int o0, int n, int w,
                                           L3<AT>* dst2 = nullptr, const G<AT>* __restrict__ B2 = nullptr) {
  for (int e = threadIdx.x; e < n * kBS; e += NT) {
    const int o = e / kBS, d = e - o * kBS;
    const int64_t src = (int64_t)(o0 + o) * w + d;
    dst[e] = d < w ? B[src] : (AT)0;
    if (B2) dst2[e] = d < w ? B2[src] : (AT)0;
  }
}

// first-direction outputs of rows [r, r + cnt) of the staged input, column o (one or two bands)
template <typename AT, typename IT, typename OT, bool TWO>
__device__ __forceinline__ void x_block(const L3<AT>* b1, const L3<AT>* b2, const L3<IT>* rows, int nin, int lo,
                                        int o, int r, int cnt, OT* out1, OT* out2, int64_t orow, int nout) {
  AT c1[kBandMax], c2[kBandMax];
#pragma unroll
  for (int d = 0; d < kBandMax; ++d) {
    c1[d] = b1[o * kBS + d];
    if (TWO) c2[d] = b2[o * kBS + d];
  }
  const bool inner = o + lo >= 0 && o + lo + kBandMax - 1 < nin;
  int jj[kBandMax];
#pragma unroll
  for (int d = 0; d < kBandMax; ++d) {
    const int j = o + lo + d;
    jj[d] = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i < cnt) {
      const L3<IT>* src = rows + (r + i) * nin;
      AT s1 = 0, s2 = 0;
      if (inner) {
        const L3<IT>* sp = src + o + lo;
#pragma unroll
        for (int d = 0; d < kBandMax; ++d) {
          const AT v = (AT)sp[d];
          s1 += c1[d] * v;
          if (TWO) s2 += c2[d] * v;
        }
      } else {
#pragma unroll
        for (int d = 0; d < kBandMax; ++d) {
          const AT v = (AT)src[jj[d]];
          s1 += c1[d] * v;
          if (TWO) s2 += c2[d] * v;
        }
      }
      out1[(orow + i) * nout + o] = (OT)s1;
      if (TWO) out2[(orow + i) * nout + o] = (OT)s2;
    }
  }
}

// pass_x with staging (the direct pass when one input row and the band do not fit)
template <int NT, typename AT, typename IT, typename OT>
__device__ void pass_x_st(int nrows, int nin, const BandDev& Bd, const IT* in, OT* out, Stg st) {
  const int nout = Bd.rows, w = Bd.w, lo = Bd.lo;
  const bool blk = w <= kBandMax;
  const int bw = al16(nout * (blk ? kBS : w) * (int)sizeof(AT));
  const int RC = (st.bytes - bw) / (nin * (int)sizeof(IT));
  if (!st.p || RC < 1) {
    pass_x<NT, AT>(nrows, nin, Bd, in, out);
    return;
  }
  L3<AT>* bs = (L3<AT>*)st.p;
  L3<IT>* rows = (L3<IT>*)(st.p + bw);
  __syncthreads();  // earlier readers of the staging area
  if (blk)
    stage_band<NT, AT>(bs, band_ptr<AT>(Bd), 0, nout, w);
  else
    stage_copy<NT>(bs, band_ptr<AT>(Bd), nout * w);
  for (int r0 = 0; r0 < nrows; r0 += RC) {
    const int rc = min(RC, nrows - r0);
    if (r0 > 0) __syncthreads();
    stage_copy<NT>(rows, in + (int64_t)r0 * nin, rc * nin);
    __syncthreads();
    if (blk) {
      const int nb = (rc + 3) / 4;
      for (int t = threadIdx.x; t < nb * nout; t += NT) {
        const int rb = t / nout, o = t - rb * nout;
        x_block<AT, IT, OT, false>(bs, bs, rows, nin, lo, o, 4 * rb, min(4, rc - 4 * rb), out, out,
                                   (int64_t)r0 + 4 * rb, nout);
      }
      continue;
    }
    for (int t = threadIdx.x; t < rc * nout; t += NT) {
      const int rr = t / nout, o = t - rr * nout;
      AT s = 0;
      for (int d = 0; d < w; ++d) {
        int j = o + lo + d;
        j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
        s += bs[o * w + d] * (AT)rows[rr * nin + j];
      }
      out[(int64_t)(r0 + rr) * nout + o] = (OT)s;
    }
  }
}

// chunk geometry of the second-direction passes: rows [o0, o0 + rc) of the output need band rows
// o0 .. o0 + rc - 1 and input rows jlo .. jhi
__device__ __forceinline__ void y_chunk(int o0, int rc, int nin, int lo, int w, int& jlo, int& jhi) {
  const int a = o0 + lo, b = o0 + rc - 1 + lo + w - 1;
  jlo = a < 0 ? 0 : (a >= nin ? nin - 1 : a);
  jhi = b < 0 ? 0 : (b >= nin ? nin - 1 : b);
}

// the 4 + kBandMax - 1 staged input values of column c that output rows oA .. oA + 3 reach
// (clamped to the input, and to the chunk's rows past its last output)
template <typename AT, typename TT>
__device__ __forceinline__ void y_column(const L3<TT>* rows, int ncols, int nin, int lo, int jlo, int jhi, int oA,
                                         int c, AT* v) {
  const int j0 = oA + lo;
  if (j0 >= 0 && j0 + 3 + kBandMax - 1 <= jhi) {
    const L3<TT>* sp = rows + (j0 - jlo) * ncols + c;
#pragma unroll
    for (int k = 0; k < 3 + kBandMax; ++k) v[k] = (AT)sp[k * ncols];
  } else {
#pragma unroll
    for (int k = 0; k < 3 + kBandMax; ++k) {
      int j = j0 + k;
      j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
      j = j > jhi ? jhi : j;
      v[k] = (AT)rows[(j - jlo) * ncols + c];
    }
  }
}

// pass_y with staging (the direct pass when w input rows and one band row do not fit)
template <int NT, typename AT, typename TT, typename ZT, typename OT>
__device__ double pass_y_st(int ncols, int nin, const BandDev& Bd, const TT* T, AT alpha, const ZT* z, AT beta,
                            bool acc, const double* scy, const double* scx, OT* out, Stg st) {
  const int nout = Bd.rows, w = Bd.w, lo = Bd.lo;
  const bool blk = w <= kBandMax;
  const int bstride = blk ? kBS : w;
  const int rowb = ncols * (int)sizeof(TT);
  const int RC = min(nout, (st.bytes - 16 - (w - 1) * rowb) / (rowb + bstride * (int)sizeof(AT)));
  if (!st.p || RC < 1) return pass_y<NT, AT>(ncols, nin, Bd, T, alpha, z, beta, acc, scy, scx, out);
  double part = 0.0;
  const int bw = al16(RC * bstride * (int)sizeof(AT));
  L3<AT>* bs = (L3<AT>*)st.p;
  L3<TT>* rows = (L3<TT>*)(st.p + bw);
  const G<AT>* __restrict__ B = band_ptr<AT>(Bd);
  __syncthreads();
  for (int o0 = 0; o0 < nout; o0 += RC) {
    const int rc = min(RC, nout - o0);
    int jlo, jhi;
    y_chunk(o0, rc, nin, lo, w, jlo, jhi);
    if (o0 > 0) __syncthreads();
    if (blk)
      stage_band<NT, AT>(bs, B, o0, rc, w);
    else
      stage_copy<NT>(bs, B + (int64_t)o0 * w, rc * w);
    stage_copy<NT>(rows, T + (int64_t)jlo * ncols, (jhi - jlo + 1) * ncols);
    __syncthreads();
    if (blk) {
      // items (block of four output rows, column), the column fastest; two items per trip, whose
      // other operands are all requested before the first output is formed
      const int items = (rc + 3) / 4 * ncols;
      for (int t0 = threadIdx.x; t0 < items; t0 += 2 * NT) {
        AT zv[2][4], av[2][4];
        double sc[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int t = t0 + q * NT, ob = t / ncols, c = t - ob * ncols;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = o0 + 4 * ob + i;
            const bool ok = t < items && o < o0 + rc;
            const int64_t ti = (int64_t)o * ncols + c;
            zv[q][i] = (z && ok) ? (AT)z[ti] : (AT)0;
            av[q][i] = (acc && ok) ? (AT)out[ti] : (AT)0;
            sc[q][i] = (scy && ok) ? gp(scy)[o] * gp(scx)[c] : 1.0;
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int t = t0 + q * NT;
          const int ob = t / ncols, c = t - ob * ncols, oA = o0 + 4 * ob;
          if (t < items) {
            AT v[3 + kBandMax];
            y_column<AT>(rows, ncols, nin, lo, jlo, jhi, oA, c, v);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int o = oA + i;
              if (o < o0 + rc) {
                const L3<AT>* bb = bs + (o - o0) * kBS;
                AT s = 0;
#pragma unroll
                for (int d = 0; d < kBandMax; ++d) s += bb[d] * v[i + d];
                AT vo = alpha * s;
                if (scy) vo *= (AT)sc[q][i];
                if (z) vo += beta * zv[q][i];
                if (acc) vo += av[q][i];
                out[(int64_t)o * ncols + c] = (OT)vo;
                part += (double)vo * (double)vo;
              }
              __builtin_amdgcn_sched_barrier(0);  // one output's band row in registers at a time
            }
          }
        }
      }
      continue;
    }
    const int base = o0 * ncols, tot = rc * ncols;
    for (int t0 = own_from<NT>(base); t0 < tot; t0 += kStU * NT) {
      // the chunk's other operands, all requested before the first output is formed
      AT zv[kStU], av[kStU];
      double sc[kStU];
#pragma unroll
      for (int u = 0; u < kStU; ++u) {
        const int t = t0 + u * NT;
        const bool ok = t < tot;
        const int o = o0 + t / ncols, c = t - (t / ncols) * ncols;
        const int64_t ti = (int64_t)base + t;
        zv[u] = (z && ok) ? (AT)z[ti] : (AT)0;
        av[u] = (acc && ok) ? (AT)out[ti] : (AT)0;
        sc[u] = (scy && ok) ? gp(scy)[o] * gp(scx)[c] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < kStU; ++u) {
        const int t = t0 + u * NT;
        if (t < tot) {
          const int oo = t / ncols, c = t - oo * ncols, o = o0 + oo;
          AT s = 0;
          for (int d = 0; d < w; ++d) {
            int j = o + lo + d;
            j = j < 0 ? 0 : (j >= nin ? nin - 1 : j);
            s += bs[oo * w + d] * (AT)rows[(j - jlo) * ncols + c];
          }
          AT v = alpha * s;
          if (scy) v *= (AT)sc[u];
          if (z) v += beta * zv[u];
          if (acc) v += av[u];
          out[(int64_t)base + t] = (OT)v;
          part += (double)v * (double)v;
        }
      }
    }
  }
  return part;
}

// pass_x2 with staging (both bands, one copy of each input row; the direct pass when they do not fit)
template <int NT, typename AT, typename IT, typename OT>
__device__ void pass_x2_st(int nrows, int nin, const BandDev& B1d, const BandDev& B2d, const IT* in, OT* out1,
                           OT* out2, Stg st) {
  const int nout = B1d.rows, w = B1d.w, lo = B1d.lo;
  const int bw = al16(nout * kBS * (int)sizeof(AT));
  const int RC = (st.bytes - 2 * bw) / (nin * (int)sizeof(IT));
  if (!st.p || RC < 1 || w > kBandMax) {
    pass_x2<NT, AT>(nrows, nin, B1d, B2d, in, out1, out2);
    return;
  }
  L3<AT>* b1 = (L3<AT>*)st.p;
  L3<AT>* b2 = (L3<AT>*)(st.p + bw);
  L3<IT>* rows = (L3<IT>*)(st.p + 2 * bw);
  __syncthreads();
  stage_band<NT, AT>(b1, band_ptr<AT>(B1d), 0, nout, w, b2, band_ptr<AT>(B2d));
  for (int r0 = 0; r0 < nrows; r0 += RC) {
    const int rc = min(RC, nrows - r0);
    if (r0 > 0) __syncthreads();
    stage_copy<NT>(rows, in + (int64_t)r0 * nin, rc * nin);
    __syncthreads();
    const int nb = (rc + 3) / 4;
    for (int t = threadIdx.x; t < nb * nout; t += NT) {
      const int rb = t / nout, o = t - rb * nout;
      x_block<AT, IT, OT, true>(b1, b2, rows, nin, lo, o, 4 * rb, min(4, rc - 4 * rb), out1, out2,
                                (int64_t)r0 + 4 * rb, nout);
    }
  }
}

// pass_y2 with staging (the direct pass when they do not fit)
template <int NT, typename AT, typename TT, typename ZT, typename OT>
__device__ double pass_y2_st(int ncols, int nin, const BandDev& B1d, const BandDev& B2d, const TT* T1,
                             const TT* T2, AT a1, AT a2, const ZT* z, AT beta, OT* out, Stg st) {
  const int nout = B1d.rows, w = B1d.w, lo = B1d.lo;
  const int rowb = ncols * (int)sizeof(TT);
  const int RC = min(nout, (st.bytes - 64 - 2 * (w - 1) * rowb) / (2 * rowb + 2 * kBS * (int)sizeof(AT)));
  if (!st.p || RC < 1 || w > kBandMax)
    return pass_y2<NT, AT>(ncols, nin, B1d, B2d, T1, T2, a1, a2, z, beta, out);
  double part = 0.0;
  const int bw = al16(RC * kBS * (int)sizeof(AT));
  L3<AT>* c1 = (L3<AT>*)st.p;
  L3<AT>* c2 = (L3<AT>*)(st.p + bw);
  const G<AT>* __restrict__ B1 = band_ptr<AT>(B1d);
  const G<AT>* __restrict__ B2 = band_ptr<AT>(B2d);
  __syncthreads();
  for (int o0 = 0; o0 < nout; o0 += RC) {
    const int rc = min(RC, nout - o0);
    int jlo, jhi;
    y_chunk(o0, rc, nin, lo, w, jlo, jhi);
    const int nr = jhi - jlo + 1;
    L3<TT>* r1 = (L3<TT>*)(st.p + 2 * bw);
    L3<TT>* r2 = (L3<TT>*)(st.p + 2 * bw + al16(nr * rowb));
    if (o0 > 0) __syncthreads();
    stage_band<NT, AT>(c1, B1, o0, rc, w, c2, B2);
    stage_copy<NT>(r1, T1 + (int64_t)jlo * ncols, nr * ncols, r2, T2 + (int64_t)jlo * ncols);
    __syncthreads();
    const int items = (rc + 3) / 4 * ncols;
    for (int t0 = threadIdx.x; t0 < items; t0 += 2 * NT) {
      AT zv[2][4];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int t = t0 + q * NT, ob = t / ncols, c = t - ob * ncols;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = o0 + 4 * ob + i;
          zv[q][i] = (z && t < items && o < o0 + rc) ? (AT)z[(int64_t)o * ncols + c] : (AT)0;
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int t = t0 + q * NT;
        const int ob = t / ncols, c = t - ob * ncols, oA = o0 + 4 * ob;
        if (t < items) {
          AT v1[3 + kBandMax], v2[3 + kBandMax];
          y_column<AT>(r1, ncols, nin, lo, jlo, jhi, oA, c, v1);
          y_column<AT>(r2, ncols, nin, lo, jlo, jhi, oA, c, v2);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = oA + i;
            if (o < o0 + rc) {
              const L3<AT>* e1 = c1 + (o - o0) * kBS;
              const L3<AT>* e2 = c2 + (o - o0) * kBS;
              AT s1 = 0, s2 = 0;
#pragma unroll
              for (int d = 0; d < kBandMax; ++d) {
                s1 += e1[d] * v1[i + d];
                s2 += e2[d] * v2[i + d];
              }
              AT vo = a1 * s1;
              if (z) vo += beta * zv[q][i];
              vo += a2 * s2;
              out[(int64_t)o * ncols + c] = (OT)vo;
              part += (double)vo * (double)vo;
            }
            __builtin_amdgcn_sched_barrier(0);  // one output's band rows in registers at a time
          }
        }
      }
    }
  }
  return part;
}

// the two terms of A_l have bands of equal shape and fit the fused passes
template <int NT>
__device__ __forceinline__ bool fusable(const InstDev& I, const LevelDev& L) {
  return L.X1.w == I.Mx2.w && L.X1.lo == I.Mx2.lo && I.My.w == I.Ky.w && I.My.lo == I.Ky.lo && L.X1.w <= kBandMax &&
         I.My.w <= kBandMax && I.Mx2.rows <= NT;
}

// out = beta z - A_l x with A_l = My (x) X1 + c Ky (x) Mx2 (temp: nin x nin scratch, may not
// alias x or out).  Returns this thread's share of ||out||^2.
// (OCC only separates the instances called from the two-workgroups-per-CU kernels, which get
// their register budget)
template <int NT, typename AT, int OCC = 1, typename XT, typename ZT, typename OT, typename TT>
__device__ double apply_A(const InstDev& I, const LevelDev& L, const XT* x, const ZT* z, OT* out, TT* tmp) {
  const int n = I.nin;
  if constexpr (sizeof(TT) == 4) {
    // FP32 temporaries: tmp is an FP64-sized slot and holds both, so the two terms of A_l take
    // one first- and one second-direction pass
    if (fusable<NT>(I, L)) {
      TT* t2 = tmp + n * n;
      pass_x2<NT, AT>(n, n, L.X1, I.Mx2, x, tmp, t2);
      __syncthreads();
      const double part =
          pass_y2<NT, AT>(n, n, I.My, I.Ky, tmp, (const TT*)t2, (AT)-1, (AT)(-L.c), z, (AT)1, out);
      __syncthreads();
      return part;
    }
  }
  pass_x<NT, AT>(n, n, L.X1, x, tmp);
  __syncthreads();
  pass_y<NT, AT>(n, n, I.My, tmp, (AT)-1, z, (AT)1, false, nullptr, nullptr, out);
  __syncthreads();
  pass_x<NT, AT>(n, n, I.Mx2, x, tmp);
  __syncthreads();
  double part = pass_y<NT, AT>(n, n, I.Ky, tmp, (AT)(-L.c), (const ZT*)nullptr, (AT)0, true, nullptr, nullptr, out);
  __syncthreads();
  return part;
}

// apply_A through LDS staging (st.p set: the vectors are in global memory).  Same roundings as
// apply_A: the fused form where apply_A fuses (FP32 temporaries, both in tmp) or where the caller
// gives a second FP64 temporary tmp2, else the four-pass form.
template <int NT, typename AT, typename XT, typename ZT, typename OT, typename TT>
__device__ double apply_A_st(const InstDev& I, const LevelDev& L, const XT* x, const ZT* z, OT* out, TT* tmp,
                             Stg st, TT* tmp2 = nullptr) {
  const int n = I.nin;
  TT* t2 = sizeof(TT) == 4 ? tmp + n * n : tmp2;
  if (t2 && fusable<NT>(I, L)) {
    pass_x2_st<NT, AT>(n, n, L.X1, I.Mx2, x, tmp, t2, st);
    __syncthreads();
    const double part = pass_y2_st<NT, AT>(n, n, I.My, I.Ky, tmp, (const TT*)t2, (AT)-1, (AT)(-L.c), z, (AT)1, out, st);
    __syncthreads();
    return part;
  }
  pass_x_st<NT, AT>(n, n, L.X1, x, tmp, st);
  __syncthreads();
  pass_y_st<NT, AT>(n, n, I.My, tmp, (AT)-1, z, (AT)1, false, nullptr, nullptr, out, st);
  __syncthreads();
  pass_x_st<NT, AT>(n, n, I.Mx2, x, tmp, st);
  __syncthreads();
  double part =
      pass_y_st<NT, AT>(n, n, I.Ky, tmp, (AT)(-L.c), (const ZT*)nullptr, (AT)0, true, nullptr, nullptr, out, st);
  __syncthreads();
  return part;
}

// ---------------------------------------------------------------------------------------
// blocked level-scheduled triangular solves
// ---------------------------------------------------------------------------------------

// Both paths solve T y = in (T = L with unit diagonal, or U), writing y (which may alias in),
// level by level over a blocked level schedule (blocks of consecutive rows, at most kDenseMax;
// a level is a set of independent blocks).

// sum over the 4 lanes of a quad with DPP lane permutes (no LDS round trip)
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
  v += dpp_mov<0xB1>(v);  // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);  // quad_perm [2, 3, 0, 1]
  return v;
}
// sum over the TG (4 or 8) lanes of a row; for 8, the quads' sums meet through row_half_mirror
// (lane i of each 8-lane group reads lane 7 - i)
template <int TG, typename T>
__device__ __forceinline__ T row_sum(T v) {
  v = quad_sum(v);
  if constexpr (TG == 8) v += dpp_mov<0x141>(v);
  return v;
}

// buffer descriptor over a table of the prefetched solve (raw, stride 0, kBufBytes long):
// a load at an offset of kBufBytes or more returns zeros without touching memory
// (the pointer is wave-uniform; reading it from the first lane puts the descriptor in scalar
// registers, as buffer instructions need)
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long a = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<void*>(p)), (short)0, (int)kBufBytes, 0x00020000);
}
constexpr int kOff = (int)0x80000000u;  // an offset past every table: the load returns zeros

template <int BYTES>
__device__ __forceinline__ void buf_load(__amdgpu_buffer_rsrc_t rs, int off, unsigned* out) {
  if constexpr (BYTES == 16) {
    typedef unsigned U4 __attribute__((ext_vector_type(4)));
    const U4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    out[0] = v.x, out[1] = v.y, out[2] = v.z, out[3] = v.w;
  } else if constexpr (BYTES == 8) {
    typedef unsigned U2 __attribute__((ext_vector_type(2)));
    const U2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    out[0] = v.x, out[1] = v.y;
  } else {
    static_assert(BYTES == 4, "unit size");
    out[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
  }
}

// Prefetched blocked triangular solve (one workgroup, TG = 4 or 8 lanes per row, up to kRowSlots
// rows per level).  Per level: phase A forms s_i = in_i - sum of the row's off-block entries times y
// (finished levels), phase B multiplies s by the row's part of the dense diagonal-block inverse.
// The tables of level l + 1 stream in while level l computes: its off-block rows are requested
// right after phase A of level l, its dense rows (and the slot metadata of level l + 2) right
// after phase B (FP32) or before phase A (FP64), so the loads overlap the barriers and the
// other phase.  Every table load is a buffer load whose unused lanes take an offset past the
// table (zeros, no memory traffic), so the loop has no divergent branches and a fixed number of
// loads in flight, and each wait covers only the data about to be used.  Off-block columns are
// stored relative to the zero word zidx, so a zeroed unit is a zero coefficient on that word.
// With WIN, y is the LDS window of the last winW grid lines (columns in the tables are window
// slots) and each solved row also goes to yg, the solution in global memory.
// widest dense row of the window mode: 128-row blocks in FP32; FP64 keeps kDenseMax (its two dense
// buffers would not fit the register budget at 128)
template <typename VT>
constexpr int kWinDense = sizeof(VT) == 4 ? kDenseWin : kDenseMax;

// DM: the widest dense row (kDenseMax, or kDenseWin for the FP32 window mode's larger blocks).
template <typename VT, bool IN_GLOBAL, int KA, int OCC, bool WIN, int DM = kDenseMax>
__device__ __noinline__ void trsv_fast(const TriDev* __restrict__ Tp, int zidx, const VT* in_g, L3<VT>* y,
                                       L3<VT>* sbuf, VT* yg) {
  constexpr int TG = Build<OCC>::TG, RW = KA * TG, V = 16 / (int)sizeof(VT);
  // dense values per lane: a row holds up to DM values after up to V - 1 of alignment
  constexpr int BCM = (DM + V - 1 + TG * V - 1) / (TG * V) * V;
  // phase B reads sbuf from the row's aligned first dense column over TG * BCM values
  static_assert(kRowSlots - 1 + TG * BCM <= kSbufWords, "sbuf too small for the dense rows");
  constexpr int WA = KA < V ? KA : V;  // off-block entries per unit
  constexpr int NU = KA / WA;          // off-block units per lane
  constexpr int ND = BCM / V;          // dense units per lane
  constexpr int VB = (int)sizeof(VT);
  typedef VT VV __attribute__((ext_vector_type(V)));
  static_assert(TG == 4 || TG == 8, "row sums over 4 or 8 lanes");
  Tp = uniform_ptr(Tp);  // the schedule header is the same for the whole workgroup
  const __amdgpu_buffer_rsrc_t rval = table_rsrc(Tp->aval), rcol = table_rsrc(Tp->acol),
                               rden = table_rsrc(Tp->dfast), rmeta = table_rsrc(Tp->meta),
                               rin = table_rsrc(in_g);
  const int R = __builtin_amdgcn_readfirstlane(Tp->R), nlev = __builtin_amdgcn_readfirstlane(Tp->nlev);
  const int r = threadIdx.x / TG, g = threadIdx.x & (TG - 1);
  const bool slot = r < R;
  const L3<VT>* yz = y + __builtin_amdgcn_readfirstlane(zidx);
  const int winW = WIN ? __builtin_amdgcn_readfirstlane(Tp->winW) : 0;
  const int winN = WIN ? __builtin_amdgcn_readfirstlane(Tp->winN) : 1;
  if ((int)((threadIdx.x & ~63) / TG) >= R) {
    // a wavefront whose row slots are all empty only keeps the barriers of the level loop
    for (int l = 0; l < nlev; ++l) {
      lds_barrier();
      lds_barrier();
    }
    return;
  }
  // slot metadata: loaded by lane 0 of each quad of the row, broadcast to the quad when its
  // level comes
  auto load_meta = [&](int l, Meta4& m) {
    unsigned u[4];
    buf_load<16>(rmeta, (g & 3) == 0 ? (slot ? 1 + l * R + r : 0) * 16 : kOff, u);
    m = Meta4{(int)u[0], (int)u[1], (int)u[2], (int)u[3]};
  };
  auto bcast = [&](Meta4& m) {
    m.row = __builtin_amdgcn_mov_dpp(m.row, 0x00, 0xF, 0xF, true);  // quad_perm [0, 0, 0, 0]
    m.bo = __builtin_amdgcn_mov_dpp(m.bo, 0x00, 0xF, 0xF, true);
    m.bqc = __builtin_amdgcn_mov_dpp(m.bqc, 0x00, 0xF, 0xF, true);
    m.na = __builtin_amdgcn_mov_dpp(m.na, 0x00, 0xF, 0xF, true);
  };
  // off-block row of slot (l, r) at RW + (l * R + r) * RW: lane g reads units g, g + TG, ... of
  // WA entries, those past the row's na entries read as zeros
  auto load_a = [&](int l, const Meta4& m, VT* av, int* ac) {
    const int base = RW + (l * R + r) * RW;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      const int e0 = (k * TG + g) * WA;
      const bool live = e0 < m.na;
      unsigned uv[WA * VB / 4], uc[WA];
      buf_load<WA * VB>(rval, live ? (base + e0) * VB : kOff, uv);
      buf_load<WA * 4>(rcol, live ? (base + e0) * 4 : kOff, uc);
#pragma unroll
      for (int e = 0; e < WA; ++e) {
        if constexpr (VB == 8)
          av[k * WA + e] = __builtin_bit_cast(double, ((unsigned long long)uv[2 * e + 1] << 32) | uv[2 * e]);
        else
          av[k * WA + e] = __builtin_bit_cast(float, uv[e]);
        ac[k * WA + e] = (int)uc[e];
      }
    }
  };
  // dense row at m.bo: lane g reads units g, g + TG, ... (bc values per lane, zeros past them),
  // and lane 0 of the quad the row's right-hand side
  auto load_b = [&](const Meta4& m, VT* bv, VT& xin) {
    // the right-hand side first: phase A needs it before phase B needs the dense row
    const bool own = g == 0 && m.row >= 0;
    if constexpr (IN_GLOBAL) {
      unsigned u[VB / 4];
      buf_load<VB>(rin, own ? m.row * VB : kOff, u);
      if constexpr (VB == 8)
        xin = __builtin_bit_cast(double, ((unsigned long long)u[1] << 32) | u[0]);
      else
        xin = __builtin_bit_cast(float, u[0]);
    } else {
      xin = ((const L3<VT>*)in_g)[own ? m.row : 0];
    }
    const int bc = m.bqc >> 16;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      unsigned u[4];
      buf_load<16>(rden, k * V < bc ? (m.bo + (k * TG + g) * V) * VB : kOff, u);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        if constexpr (VB == 8)
          bv[k * V + e] = __builtin_bit_cast(double, ((unsigned long long)u[2 * e + 1] << 32) | u[2 * e]);
        else
          bv[k * V + e] = __builtin_bit_cast(float, u[e]);
      }
    }
  };
  auto phase_a = [&](const VT* av, const int* ac, int row, VT xin) {
    VT s = 0;
#pragma unroll
    for (int j = 0; j < KA; ++j) s += av[j] * yz[ac[j]];
    s = row_sum<TG>(s);
    if (g == 0 && row >= 0) sbuf[r] = xin - s;
  };
  // sbuf beyond the level's rows holds finite values, met by zero coefficients
  auto phase_b = [&](const VT* bv, const Meta4& m) {
    VT s = 0;
    const L3<VV>* sp = (const L3<VV>*)(sbuf + (m.bqc & 0xffff));
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      const VV sv = sp[k * TG + g];
#pragma unroll
      for (int e = 0; e < V; ++e) s += bv[k * V + e] * sv[e];
    }
    s = row_sum<TG>(s);
    if (g == 0 && m.row >= 0) {
      if constexpr (WIN) {
        const int line = m.row / winN;
        y[(line % winW) * winN + (m.row - line * winN)] = s;
        ((G<VT>*)yg)[m.row] = s;
      } else {
        y[m.row] = s;
      }
    }
  };
  if constexpr (sizeof(VT) == 4 || OCC == 3) {
    // FP32, and the 1024-thread build (one buffer per table).  Level l starts with its off-block rows (av, ac), dense row
    // (bv, xin) and broadcast metadata (C) loaded or in flight, and level l + 1's metadata record
    // in N.  Level l + 1's off-block rows are requested after phase A of level l, its dense row
    // after phase B; the scheduling barriers keep those requests where they are, so that each
    // wait covers only the data about to be used.
    VT av[KA], bv[BCM], xin;
    int ac[KA];
    Meta4 C, N;
    load_meta(0, C);
    load_meta(1, N);
    __builtin_amdgcn_sched_barrier(0);
    bcast(C);
    load_a(0, C, av, ac);
    __builtin_amdgcn_sched_barrier(0);
    load_b(C, bv, xin);
    __builtin_amdgcn_sched_barrier(0);
    for (int l = 0; l < nlev; ++l) {
      phase_a(av, ac, C.row, xin);
      __builtin_amdgcn_sched_barrier(0);
      bcast(N);
      load_a(l + 1, N, av, ac);
      lds_barrier();
      phase_b(bv, C);
      __builtin_amdgcn_sched_barrier(0);
      Meta4 N2;
      load_meta(l + 2, N2);
      load_b(N, bv, xin);
      C = N;
      N = N2;
      lds_barrier();
    }
  } else {
    // FP64 with 512 threads (dense rows twice as wide: two dense buffers, so that the next level's dense row
    // streams in during phase A rather than holding up the barrier after phase B).  The loop is
    // unrolled by two: at even level l, M0 (broadcast), bv0, x0 and av/ac hold its data and M1
    // level l + 1's metadata record.
    VT av[KA], bv0[BCM], bv1[BCM], x0, x1;
    int ac[KA];
    Meta4 M0, M1;
    load_meta(0, M0);
    load_meta(1, M1);
    __builtin_amdgcn_sched_barrier(0);
    bcast(M0);
    load_b(M0, bv0, x0);
    __builtin_amdgcn_sched_barrier(0);
    load_a(0, M0, av, ac);
    __builtin_amdgcn_sched_barrier(0);
    for (int l = 0; l < nlev; l += 2) {
      {  // even level l
        const Meta4 m = M0;
        bcast(M1);
        load_b(M1, bv1, x1);
        load_meta(l + 2, M0);
        phase_a(av, ac, m.row, x0);
        lds_barrier();
        load_a(l + 1, M1, av, ac);
        phase_b(bv0, m);
        lds_barrier();
      }
      if (l + 1 >= nlev) break;
      {  // odd level l + 1
        const Meta4 m = M1;
        bcast(M0);
        load_b(M0, bv0, x0);
        load_meta(l + 3, M1);
        phase_a(av, ac, m.row, x1);
        lds_barrier();
        load_a(l + 2, M0, av, ac);
        phase_b(bv1, m);
        lds_barrier();
      }
    }
  }
}


// Window-mode solve over slab tables (TriDev::dch > 0; 512 threads, 4 lanes per row, 128 row slots).
// A level's dense rows lie contiguous in a slab of dch x 8 KB, which the whole workgroup copies into
// the LDS area dst with one 16-byte load per lane per 8 KB, so the dense rows cost no loads for their
// padding lanes; the off-block columns are 16 bits, each lane's KA of them contiguous.  A level of
// the window mode is bound by the CU's vector-memory path (instructions, padding lanes included, and
// bytes), so these take about a third fewer instructions.  The off-block rows are requested one level
// ahead, the right-hand sides two levels ahead, the metadata three, and the slabs two levels ahead in
// FP32 (two register sets, even and odd levels) and one in FP64 (slabs twice as large).  The
// arithmetic is trsv_fast's, in the same order.
template <typename VT, int KA>
__device__ __noinline__ void trsv_slab(const TriDev* __restrict__ Tp, int zidx, const VT* in_g, L3<VT>* y,
                                       L3<VT>* sbuf, VT* yg, L3<VT>* dst) {
  constexpr int VB = (int)sizeof(VT), TG = 4, RW = KA * TG, V = 16 / VB, WA = KA < V ? KA : V, NU = KA / WA;
  constexpr int CB = KA * 2, DCH = kDchOf<VT>;
  // register sets of slabs in flight: two (two levels ahead) in FP32; one (one level ahead) in FP64,
  // whose slabs are twice as large
  constexpr int SETS = VB == 4 ? 2 : 1;
  constexpr int BCM = (kDenseWin + V - 1 + TG * V - 1) / (TG * V) * V, ND = BCM / V;
  static_assert(kRowSlots - 1 + TG * BCM <= kSbufWords, "sbuf too small for the dense rows");
  typedef VT VV __attribute__((ext_vector_type(V)));
  typedef unsigned U4 __attribute__((ext_vector_type(4)));
  Tp = uniform_ptr(Tp);
  const __amdgpu_buffer_rsrc_t rval = table_rsrc(Tp->aval), rc16 = table_rsrc(Tp->acol16),
                               rden = table_rsrc(Tp->dfast), rmeta = table_rsrc(Tp->meta), rin = table_rsrc(in_g);
  const int R = __builtin_amdgcn_readfirstlane(Tp->R), nlev = __builtin_amdgcn_readfirstlane(Tp->nlev);
  const int dch = __builtin_amdgcn_readfirstlane(Tp->dch), lsv = __builtin_amdgcn_readfirstlane(Tp->lsv);
  const int winW = __builtin_amdgcn_readfirstlane(Tp->winW), winN = __builtin_amdgcn_readfirstlane(Tp->winN);
  const int r = threadIdx.x / TG, g = threadIdx.x & (TG - 1);
  const L3<VT>* yz = y + __builtin_amdgcn_readfirstlane(zidx);
  auto load_meta = [&](int l, Meta4& m) {
    unsigned u[4];
    buf_load<16>(rmeta, g == 0 ? (1 + l * R + r) * 16 : kOff, u);
    m = Meta4{(int)u[0], (int)u[1], (int)u[2], (int)u[3]};
  };
  auto bcast = [&](Meta4& m) {
    m.row = __builtin_amdgcn_mov_dpp(m.row, 0x00, 0xF, 0xF, true);  // quad_perm [0, 0, 0, 0]
    m.bo = __builtin_amdgcn_mov_dpp(m.bo, 0x00, 0xF, 0xF, true);
    m.bqc = __builtin_amdgcn_mov_dpp(m.bqc, 0x00, 0xF, 0xF, true);
    m.na = __builtin_amdgcn_mov_dpp(m.na, 0x00, 0xF, 0xF, true);
  };
  auto load_a = [&](int l, const Meta4& m, VT* av, int* ac) {
    const int base = RW + (l * R + r) * RW;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      const int e0 = (k * TG + g) * WA;
      unsigned uv[WA * VB / 4];
      buf_load<WA * VB>(rval, e0 < m.na ? (base + e0) * VB : kOff, uv);
#pragma unroll
      for (int e = 0; e < WA; ++e) {
        if constexpr (VB == 8)
          av[k * WA + e] = __builtin_bit_cast(double, ((unsigned long long)uv[2 * e + 1] << 32) | uv[2 * e]);
        else
          av[k * WA + e] = __builtin_bit_cast(float, uv[e]);
      }
    }
    // lane g's columns (k * WA + e order) at (base + g * KA) * 2 bytes, zero past the row's entries
    const bool live = l < nlev;
    const int c0 = (base + g * KA) * 2;
    unsigned uc[(CB + 3) / 4];
#pragma unroll
    for (int q = 0; q < CB / 16; ++q) buf_load<16>(rc16, live ? c0 + q * 16 : kOff, uc + q * 4);
    if constexpr (CB % 16 != 0) buf_load<CB % 16>(rc16, live ? c0 + CB / 16 * 16 : kOff, uc + CB / 16 * 4);
#pragma unroll
    for (int j = 0; j < KA; ++j) ac[j] = (int)(short)(unsigned short)(uc[j / 2] >> (16 * (j % 2)));
  };
  // the row's right-hand side, by the lane that writes its result (it holds the raw record)
  auto load_x = [&](const Meta4& m, VT& xin) {
    unsigned u[VB / 4];
    buf_load<VB>(rin, g == 0 && m.row >= 0 ? m.row * VB : kOff, u);
    if constexpr (VB == 8)
      xin = __builtin_bit_cast(double, ((unsigned long long)u[1] << 32) | u[0]);
    else
      xin = __builtin_bit_cast(float, u[0]);
  };
  auto load_d = [&](int l, U4* dr) {
    const int b0 = (kSlab0 + l * lsv) * VB + (int)threadIdx.x * 16;
    const bool live = l < nlev;
#pragma unroll
    for (int c = 0; c < DCH; ++c) {
      unsigned u[4];
      buf_load<16>(rden, live && c < dch ? b0 + c * kChunkBytes : kOff, u);
      dr[c] = U4{u[0], u[1], u[2], u[3]};
    }
  };
  auto store_d = [&](const U4* dr) {
#pragma unroll
    for (int c = 0; c < DCH; ++c) ((L3<U4>*)dst)[c * (kChunkBytes / 16) + threadIdx.x] = dr[c];
  };
  auto phase_a = [&](const VT* av, const int* ac, int row, VT xin) {
    VT s = 0;
#pragma unroll
    for (int j = 0; j < KA; ++j) s += av[j] * yz[ac[j]];
    s = row_sum<TG>(s);
    if (g == 0 && row >= 0) sbuf[r] = xin - s;
  };
  auto phase_b = [&](const Meta4& m, int l) {
    VT s = 0;
    const L3<VV>* sp = (const L3<VV>*)(sbuf + (m.bqc & 0xffff));
    const int rel = m.row >= 0 ? m.bo - (kSlab0 + l * lsv) : 0;  // the row's offset in its slab
    const L3<VV>* dp = (const L3<VV>*)(dst + rel);
    const int bc = m.bqc >> 16;
#pragma unroll 3
    for (int k = 0; k < ND; ++k) {
      const VV sv = sp[k * TG + g];
      const bool on = k * V < bc;
      const VV dv = dp[on ? k * TG + g : 0];
#pragma unroll
      for (int e = 0; e < V; ++e) s += (on ? dv[e] : (VT)0) * sv[e];
    }
    s = row_sum<TG>(s);
    if (g == 0 && m.row >= 0) {
      const int line = m.row / winN;
      y[(line % winW) * winN + (m.row - line * winN)] = s;
      ((G<VT>*)yg)[m.row] = s;
    }
  };
  // level l starts with C and N (levels l and l + 1, broadcast) and N2 (level l + 2, raw), its own
  // off-block rows, and its right-hand side and slab in register set l mod 2 (level l + 1's in the
  // other set)
  VT av[KA], x0, x1;
  int ac[KA];
  U4 d0[DCH], d1[SETS == 2 ? DCH : 1];
  Meta4 C, N, N2;
  load_meta(0, C);
  load_meta(1, N);
  load_meta(2, N2);
  __builtin_amdgcn_sched_barrier(0);
  load_x(C, x0);
  load_x(N, x1);
  bcast(C);
  load_a(0, C, av, ac);
  __builtin_amdgcn_sched_barrier(0);
  load_d(0, d0);
  if constexpr (SETS == 2) load_d(1, d1);
  __builtin_amdgcn_sched_barrier(0);
  // one level: phase A, its slab into LDS, level l + 1's off-block rows requested, phase B from LDS,
  // then level l + 3's metadata and level l + 2's right-hand side and slab
  auto level = [&](int l, VT& xin, U4* dr) {
    phase_a(av, ac, C.row, xin);
    store_d(dr);
    __builtin_amdgcn_sched_barrier(0);
    bcast(N);
    load_a(l + 1, N, av, ac);
    lds_barrier();
    phase_b(C, l);
    __builtin_amdgcn_sched_barrier(0);
    Meta4 N3;
    load_meta(l + 3, N3);
    load_x(N2, xin);
    load_d(l + SETS, dr);
    C = N;
    N = N2;
    N2 = N3;
    lds_barrier();
  };
  for (int l = 0; l < nlev; l += 2) {
    level(l, x0, d0);
    if (l + 1 >= nlev) break;
    level(l + 1, x1, SETS == 2 ? d1 : d0);
  }
}

// General path (any schedule, y in LDS or global): same two phases with loops, full barriers.
template <typename VT, int NT>
__device__ void trsv_general(const TriDev& T, const VT* in, VT* y, VT* sbuf) {
  constexpr int GA = 8, GB = 8;
  const G<VT>* __restrict__ ov = gp((const VT*)T.ov);
  const G<VT>* __restrict__ dv = gp((const VT*)T.dval);
  const G<int>* __restrict__ lev_ptr = gp(T.lev_ptr);
  const G<int>* __restrict__ rowv = gp(T.row);
  const G<int>* __restrict__ orp = gp(T.orp);
  const G<int>* __restrict__ oci = gp(T.oci);
  const G<int>* __restrict__ dq0 = gp(T.dq0);
  const G<int>* __restrict__ dcnt = gp(T.dcnt);
  const G<int64_t>* __restrict__ doff = gp(T.doff);
  const int nlev = T.nlev;
  const int ga = threadIdx.x & (GA - 1), gb = threadIdx.x & (GB - 1);
  for (int l = 0; l < nlev; ++l) {
    const int q0 = lev_ptr[l], q1 = lev_ptr[l + 1];
    for (int q = q0 + threadIdx.x / GA; q < q1; q += NT / GA) {
      const int i = rowv[q];
      VT s = 0;
      for (int k = orp[q] + ga; k < orp[q + 1]; k += GA) s += ov[k] * y[oci[k]];
      s = group_sum<GA>(s);
      if (ga == 0) sbuf[q - q0] = in[i] - s;
    }
    __syncthreads();
    for (int q = q0 + threadIdx.x / GB; q < q1; q += NT / GB) {
      const int c0 = dq0[q], cn = dcnt[q];
      const G<VT>* __restrict__ dr = dv + doff[q];
      VT s = 0;
      for (int c = gb; c < cn; c += GB) s += dr[c] * sbuf[c0 + c];
      s = group_sum<GB>(s);
      if (gb == 0) y[rowv[q]] = s;
    }
    __syncthreads();
  }
}

// win: the LDS window of the triangular solves when y is in global memory (null: none)
template <typename VT, bool YLDS, bool IN_GLOBAL, int OCC>
__device__ __forceinline__ void trsv(const TriDev& T, int ka, int zidx, const VT* in, VT* y, VT* sbuf, VT* win,
                                     int zwin, Stg st = Stg{}) {
  L3<VT>* sl = (L3<VT>*)sbuf;
  if (YLDS && T.fast) {
    L3<VT>* yl = (L3<VT>*)y;
    if (ka <= 2)
      trsv_fast<VT, IN_GLOBAL, 2, OCC, false>(&T, zidx, in, yl, sl, nullptr);
    else if (ka <= 4)
      trsv_fast<VT, IN_GLOBAL, 4, OCC, false>(&T, zidx, in, yl, sl, nullptr);
    else if (ka <= 8)
      trsv_fast<VT, IN_GLOBAL, 8, OCC, false>(&T, zidx, in, yl, sl, nullptr);
    else if (ka <= 12)
      trsv_fast<VT, IN_GLOBAL, 12, OCC, false>(&T, zidx, in, yl, sl, nullptr);
    else
      trsv_fast<VT, IN_GLOBAL, 16, OCC, false>(&T, zidx, in, yl, sl, nullptr);
  } else if (!YLDS && IN_GLOBAL && (OCC == 1 || OCC == 2) && win && T.fast && T.winW > 0) {
    L3<VT>* wl = (L3<VT>*)win;
    bool slab = false;
    if constexpr (OCC == 1) {
      // slab tables, with the band-pass staging area as the slabs' LDS area
      if (T.dch > 0 && T.R * 4 == Build<OCC>::NT && st.p && st.bytes >= kDchOf<VT> * kChunkBytes) {
        slab = true;
        L3<VT>* sf = (L3<VT>*)sbuf;
        L3<VT>* ds = (L3<VT>*)st.p;
        if (ka <= 2)
          trsv_slab<VT, 2>(&T, zwin, in, wl, sf, y, ds);
        else if (ka <= 4)
          trsv_slab<VT, 4>(&T, zwin, in, wl, sf, y, ds);
        else if (ka <= 8)
          trsv_slab<VT, 8>(&T, zwin, in, wl, sf, y, ds);
        else if (ka <= 12)
          trsv_slab<VT, 12>(&T, zwin, in, wl, sf, y, ds);
        else
          trsv_slab<VT, 16>(&T, zwin, in, wl, sf, y, ds);
      }
    }
    if (!slab && sizeof(VT) == 8 && T.dch > 0) {
      // FP64 slab tables hold dense rows wider than the register path takes: the general path
      slab = true;
      trsv_general<VT, Build<OCC>::NT>(T, in, y, sbuf);
    }
    if (!slab) {
      if (ka <= 2)
        trsv_fast<VT, true, 2, OCC, true, kWinDense<VT>>(&T, zwin, in, wl, sl, y);
      else if (ka <= 4)
        trsv_fast<VT, true, 4, OCC, true, kWinDense<VT>>(&T, zwin, in, wl, sl, y);
      else if (ka <= 8)
        trsv_fast<VT, true, 8, OCC, true, kWinDense<VT>>(&T, zwin, in, wl, sl, y);
      else if (ka <= 12)
        trsv_fast<VT, true, 12, OCC, true, kWinDense<VT>>(&T, zwin, in, wl, sl, y);
      else
        trsv_fast<VT, true, 16, OCC, true, kWinDense<VT>>(&T, zwin, in, wl, sl, y);
    }
  } else {
    trsv_general<VT, Build<OCC>::NT>(T, in, y, sbuf);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// exact p = 1 solve: fast diagonalisation c = V diag-solve(V^T c), one symmetric tridiagonal
// system per mode of the second direction (Thomas, precomputed LDL^T).  c1 in / out, c2 temp.
// ---------------------------------------------------------------------------------------
// Dense transforms of the fast diagonalisation on the matrix cores (FP64 MFMA, 16 x 16 x 4):
//   out(a, x) = sum_b W(a, b) In(b, x)   for a, x < n1,
// W(a, b) = V[b][a] (WT) or V[a][b]; In(b, x) = in[x][b] (IT) or in[b][x]; the result is stored at
// out[x][a] (OT) or out[a][x].  Workgroup tiles of 128 x TX outputs (TX = 16 BC times the waves / 4),
// each wave a 32 x 16 BC part (2 x BC blocks of 16 x 16).  With an LDS staging area of
// kStageDoubles the contraction runs in chunks of KC = 8 staged in LDS (with BC = 4 the next chunk's
// loads are held in registers while the current one is multiplied); without one each wave reads its
// operand fragments from global memory, one step of 4 ahead.  Every output is accumulated over b in
// increasing steps of 4 in every variant (steps past n1 add zero products), so all of them give
// the same values.
typedef double d4v __attribute__((ext_vector_type(4)));
// operand and result layouts of v_mfma_f64_16x16x4f64 for lane l: A[l % 16][l / 16],
// B[l / 16][l % 16], element r of D: D[l / 16 + 4 r][l % 16]
__device__ __forceinline__ d4v mfma_f64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <bool WT>
__device__ __forceinline__ double w_at(const G<double>* __restrict__ V, int n1, int a, int b) {
  return (a < n1 && b < n1) ? (WT ? V[b * n1 + a] : V[a * n1 + b]) : 0.0;
}
template <bool IT>
__device__ __forceinline__ double in_at(const double* in, int n1, int b, int x) {
  return (b < n1 && x < n1) ? (IT ? in[x * n1 + b] : in[b * n1 + x]) : 0.0;
}

template <int NT, int BC, bool WT, bool IT, bool OT>
__device__ void coarse_gemm(int n1, const G<double>* __restrict__ V, const double* in, double* out, double* stage) {
  constexpr int NW = NT / 64, WC = NW / 4, TA = 128, TX = WC * 16 * BC, KC = 8;
  static_assert(NW % 4 == 0 && KC * (TA + TX) <= kStageDoubles, "tile shape");
  // the next chunk is held in registers only in the builds with the full register budget (BC = 4)
  constexpr bool PF = BC >= 4;
  constexpr int EW = PF ? KC * TA / NT : 1, EI = PF ? KC * TX / NT : 1;  // chunk elements per thread
  static_assert(!PF || (EW * NT == KC * TA && EI * NT == KC * TX), "chunk split");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = wv % 4, wc = wv / 4, li = lane & 15, lk = lane >> 4;
  L3<double>* ws = (L3<double>*)stage;  // [KC][TA]
  L3<double>* is = ws + KC * TA;        // [KC][TX]
  for (int a0 = 0; a0 < n1; a0 += TA)
    for (int x0 = 0; x0 < n1; x0 += TX) {
      d4v acc[2][BC];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < BC; ++cb) acc[rb][cb] = d4v{0.0, 0.0, 0.0, 0.0};
      const int ra = a0 + wr * 32 + li, cx = x0 + wc * 16 * BC + li;
      if (stage) {
        // element e of a chunk: W part kk = e / TA, aa = e % TA (WT: consecutive a are consecutive in
        // memory) or kk = e % KC, aa = e / KC; In part likewise with IT
        double pw[EW], pi[EI];
        auto fetch = [&](int k0) {
#pragma unroll
          for (int j = 0; j < EW; ++j) {
            const int e = threadIdx.x + j * NT;
            const int kk = WT ? e / TA : e % KC, aa = WT ? e % TA : e / KC;
            pw[j] = w_at<WT>(V, n1, a0 + aa, k0 + kk);
          }
#pragma unroll
          for (int j = 0; j < EI; ++j) {
            const int e = threadIdx.x + j * NT;
            const int kk = IT ? e % KC : e / TX, xx = IT ? e / KC : e % TX;
            pi[j] = in_at<IT>(in, n1, k0 + kk, x0 + xx);
          }
        };
        if constexpr (PF) fetch(0);
        for (int k0 = 0; k0 < n1; k0 += KC) {
          __syncthreads();  // the previous chunk has been consumed
          if constexpr (PF) {
#pragma unroll
            for (int j = 0; j < EW; ++j) {
              const int e = threadIdx.x + j * NT;
              const int kk = WT ? e / TA : e % KC, aa = WT ? e % TA : e / KC;
              ws[kk * TA + aa] = pw[j];
            }
#pragma unroll
            for (int j = 0; j < EI; ++j) {
              const int e = threadIdx.x + j * NT;
              const int kk = IT ? e % KC : e / TX, xx = IT ? e / KC : e % TX;
              is[kk * TX + xx] = pi[j];
            }
          } else {
            for (int e = threadIdx.x; e < KC * TA; e += NT) {
              const int kk = WT ? e / TA : e % KC, aa = WT ? e % TA : e / KC;
              ws[kk * TA + aa] = w_at<WT>(V, n1, a0 + aa, k0 + kk);
            }
            for (int e = threadIdx.x; e < KC * TX; e += NT) {
              const int kk = IT ? e % KC : e / TX, xx = IT ? e / KC : e % TX;
              is[kk * TX + xx] = in_at<IT>(in, n1, k0 + kk, x0 + xx);
            }
          }
          __syncthreads();
          if constexpr (PF)
            if (k0 + KC < n1) fetch(k0 + KC);
#pragma unroll
          for (int ks = 0; ks < KC; ks += 4) {
            double fa[2], fb[BC];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) fa[rb] = ws[(ks + lk) * TA + wr * 32 + rb * 16 + li];
#pragma unroll
            for (int cb = 0; cb < BC; ++cb) fb[cb] = is[(ks + lk) * TX + wc * 16 * BC + cb * 16 + li];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
              for (int cb = 0; cb < BC; ++cb) acc[rb][cb] = mfma_f64(fa[rb], fb[cb], acc[rb][cb]);
          }
        }
      } else {
        double fa[2], fb[BC];
        auto frag = [&](int k0) {
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) fa[rb] = w_at<WT>(V, n1, ra + rb * 16, k0 + lk);
#pragma unroll
          for (int cb = 0; cb < BC; ++cb) fb[cb] = in_at<IT>(in, n1, k0 + lk, cx + cb * 16);
        };
        frag(0);
        for (int k0 = 0; k0 < n1; k0 += 4) {
          const double ca0 = fa[0], ca1 = fa[1];
          double cbv[BC];
#pragma unroll
          for (int cb = 0; cb < BC; ++cb) cbv[cb] = fb[cb];
          if (k0 + 4 < n1) frag(k0 + 4);
#pragma unroll
          for (int cb = 0; cb < BC; ++cb) {
            acc[0][cb] = mfma_f64(ca0, cbv[cb], acc[0][cb]);
            acc[1][cb] = mfma_f64(ca1, cbv[cb], acc[1][cb]);
          }
        }
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < BC; ++cb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a = a0 + wr * 32 + rb * 16 + lk + 4 * r, x = x0 + wc * 16 * BC + cb * 16 + li;
            if (a < n1 && x < n1) out[OT ? x * n1 + a : a * n1 + x] = acc[rb][cb][r];
          }
    }
}

// (G + c lam_k H) solves of one n1 x n1 grid by fast diagonalisation with eigenvectors V (n1 x n1,
// V[iy][k]) and the Thomas data tl / tdinv of the modes, stored by node (tl[i * n1 + k]): c1 in / out,
// c2 temporary (the modes' values, node-major: c2[ix * n1 + k]); stage: an LDS staging area of
// kStageDoubles for the transforms (null: none).  BC: the transforms' wave tile width in blocks.
template <int NT, int BC = 2>
__device__ __forceinline__ void fdm_solve(int n1, const double* Vp, const double* tlp, const double* tdp, double* c1,
                                          double* c2, double* stage = nullptr) {
  const G<double>* __restrict__ V = gp(Vp);
  // c2[ix][k] = sum_iy V[iy][k] c1[iy][ix]
  coarse_gemm<NT, BC, true, false, true>(n1, V, c1, c2, stage);
  __syncthreads();
  // one thread per mode k, the nodes in sequence; consecutive threads read consecutive words.  The
  // coefficients and values are loaded 8 nodes at a time, ahead of the recurrence, so their latency
  // is paid once per chunk; results are stored after the chunk
  for (int k = threadIdx.x; k < n1; k += NT) {
    constexpr int CH = 8;
    const G<double>* __restrict__ tl = gp(tlp);
    const G<double>* __restrict__ td = gp(tdp);
    double yp = 0.0;
    for (int i0 = 0; i0 < n1; i0 += CH) {
      double a[CH], b[CH], v[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int i = i0 + u < n1 ? i0 + u : n1 - 1;
        a[u] = tl[i * n1 + k];
        b[u] = td[i * n1 + k];
        v[u] = c2[i * n1 + k];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int i = i0 + u;
        const double yv = v[u] - (i > 0 ? a[u] * yp : 0.0);
        v[u] = yv * b[u];
        yp = i < n1 ? yv : yp;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (i0 + u < n1) c2[(i0 + u) * n1 + k] = v[u];
    }
    double xn = 0.0;
    for (int i1 = n1 - 1; i1 >= 0; i1 -= CH) {
      double a[CH], v[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int i = i1 - u + 1;  // multiplier l_{i+1} for row i = i1 - u
        a[u] = (i >= 1 && i < n1) ? tl[i * n1 + k] : 0.0;
        v[u] = c2[(i1 - u >= 0 ? i1 - u : 0) * n1 + k];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int i = i1 - u;
        if (i >= 0) {
          xn = (i == n1 - 1) ? v[u] : v[u] - a[u] * xn;
          v[u] = xn;
        }
      }
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (i1 - u >= 0) c2[(i1 - u) * n1 + k] = v[u];
    }
  }
  __syncthreads();
  // c1[iy][ix] = sum_k V[iy][k] c2[ix][k]
  coarse_gemm<NT, BC, false, true, false>(n1, V, c2, c1, stage);
  __syncthreads();
}

// exact p = 1 solve of A_{h,1} = M1 + c K1 (c1 in / out, c2 temporary)
template <int NT, int BC>
__device__ __forceinline__ void coarse_solve(const InstDev& I, const LevelDev& L, double* c1, double* c2,
                                             double* stage) {
  fdm_solve<NT, BC>(I.n1, I.V, L.tl, L.tdinv, c1, c2, stage);
}

// ---------------------------------------------------------------------------------------
// p = 1 solve by one h-multigrid W-cycle (Sec. 4, the paragraph after step 5): four-colour
// Gauss-Seidel pre- and post-smoothing, residual restricted by R = P^T, two W-cycles on the next
// level (one solve at the coarsest), prolongation of the correction by the canonical P.
// Grids of h-level k are n1 x n1 interior nodes, first index fastest.
// ---------------------------------------------------------------------------------------

// the nine stencil coefficients of A_k at node (iy, ix): a[dy + 1][dx + 1]
__device__ __forceinline__ void hmg_stencil(const G<double>* __restrict__ bd, int n1, int iy, int ix, double c,
                                            double a[3][3]) {
  const G<double>* Mx = bd + 3 * ix;
  const G<double>* Kx = bd + 3 * (n1 + ix);
  const G<double>* M2 = bd + 3 * (2 * n1 + ix);
  const G<double>* My = bd + 3 * (3 * n1 + iy);
  const G<double>* Ky = bd + 3 * (4 * n1 + iy);
  double xa[3], xb[3], ya[3], yb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xa[d] = Mx[d] + c * Kx[d];
    xb[d] = c * M2[d];
    ya[d] = My[d];
    yb[d] = Ky[d];
  }
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) a[dy][dx] = ya[dy] * xa[dx] + yb[dy] * xb[dx];
}

// sum over the off-centre stencil entries of a * x around (iy, ix) (neighbours outside the grid
// have zero coefficients: the band rows hold zeros there)
__device__ __forceinline__ double hmg_offsum(const double a[3][3], const double* x, int n1, int iy, int ix) {
  double s = 0.0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      if (dy == 0 && dx == 0) continue;
      const int jy = iy + dy, jx = ix + dx;
      if (jy >= 0 && jy < n1 && jx >= 0 && jx < n1) s += a[dy + 1][dx + 1] * x[jy * n1 + jx];
    }
  return s;
}

// one Gauss-Seidel sweep in the four-colour order of the 9-point stencil (colour of node (ix, iy) is
// (ix mod 2) + 2 (iy mod 2)): colours 0..3 (fwd) or 3..0; nodes of one colour never couple
template <int NT>
__device__ __forceinline__ void hmg_gs(const double* band, int n1, double c, const double* b, double* x, bool fwd) {
  const G<double>* __restrict__ bd = gp(band);
  for (int cc = 0; cc < 4; ++cc) {
    const int col = fwd ? cc : 3 - cc;
    const int ox = col & 1, oy = col >> 1;
    const int nx = (n1 - ox + 1) >> 1, ny = (n1 - oy + 1) >> 1;
    for (int t = threadIdx.x; t < nx * ny; t += NT) {
      const int iy = 2 * (t / nx) + oy, ix = 2 * (t % nx) + ox;
      double a[3][3];
      hmg_stencil(bd, n1, iy, ix, c, a);
      x[iy * n1 + ix] = (b[iy * n1 + ix] - hmg_offsum(a, x, n1, iy, ix)) / a[1][1];
    }
    __syncthreads();
  }
}

// r = b - A_k x on h-level k, then the restriction bc = R r onto level k + 1 (coarse node J sits on
// fine node 2J + 1, its hat has weights 1/2, 1, 1/2 on fine nodes 2J, 2J + 1, 2J + 2), xc = 0
template <int NT>
__device__ __forceinline__ void hmg_restrict(const double* band, int n1, double c, const double* b, const double* x, double* r,
                             int n1c, double* bc, double* xc) {
  const G<double>* __restrict__ bd = gp(band);
  for (int t = threadIdx.x; t < n1 * n1; t += NT) {
    const int iy = t / n1, ix = t - iy * n1;
    double a[3][3];
    hmg_stencil(bd, n1, iy, ix, c, a);
    r[t] = b[t] - (a[1][1] * x[t] + hmg_offsum(a, x, n1, iy, ix));
  }
  __syncthreads();
  const double w[3] = {0.5, 1.0, 0.5};
  for (int t = threadIdx.x; t < n1c * n1c; t += NT) {
    const int jy = t / n1c, jx = t - jy * n1c;
    double s = 0.0;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      double sx = 0.0;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) sx += w[dx] * r[(2 * jy + dy) * n1 + 2 * jx + dx];
      s += w[dy] * sx;
    }
    bc[t] = s;
    xc[t] = 0.0;
  }
  __syncthreads();
}

// x += P xc: fine node i (0-based) takes coarse node (i - 1) / 2 with weight 1 when i is odd, and
// coarse nodes i / 2 - 1 and i / 2 with weights 1/2 when i is even (those that exist)
template <int NT>
__device__ __forceinline__ void hmg_prolong(int n1, int n1c, const double* xc, double* x) {
  for (int t = threadIdx.x; t < n1 * n1; t += NT) {
    const int iy = t / n1, ix = t - iy * n1;
    int jy[2], jx[2];
    double wy[2], wx[2];
    if (iy & 1) { jy[0] = (iy - 1) >> 1; wy[0] = 1.0; jy[1] = 0; wy[1] = 0.0; }
    else { jy[0] = (iy >> 1) - 1; wy[0] = 0.5; jy[1] = iy >> 1; wy[1] = 0.5; }
    if (ix & 1) { jx[0] = (ix - 1) >> 1; wx[0] = 1.0; jx[1] = 0; wx[1] = 0.0; }
    else { jx[0] = (ix >> 1) - 1; wx[0] = 0.5; jx[1] = ix >> 1; wx[1] = 0.5; }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const bool ok = wy[u] != 0.0 && wx[v] != 0.0 && jy[u] >= 0 && jy[u] < n1c && jx[v] >= 0 && jx[v] < n1c;
        if (ok) s += wy[u] * wx[v] * xc[jy[u] * n1c + jx[v]];
      }
    x[t] += s;
  }
  __syncthreads();
}

// x0 = W-cycle(A_0, b0) from x0 = 0; the recursion W(k) = GS, restrict, W(k+1) twice (once when
// k + 1 is the coarsest level, which is solved exactly), prolong, GS backwards, run as a loop over
// the levels with one bit per level recording whether its first W(k+1) is done.  hw: scratch of
// HmgDev::words doubles (residual temporary, then b_k, x_k of the coarser levels)
template <int NT>
__device__ __forceinline__ void hmg_wcycle(const InstDev& I, const LevelDev& L, const double* b0, double* x0, double* hw) {
  const HmgDev& H = I.hmg;
  const int last = H.nh - 1;
  const double c = L.c;
  double* rt = hw;
  for (int i = threadIdx.x; i < H.n1[0] * H.n1[0]; i += NT) x0[i] = 0.0;
  __syncthreads();
  unsigned once = 0;  // bit k: the first W(k + 1) of level k's current activation has returned
  int k = 0;
  bool down = true;
  for (;;) {
    const int n1 = H.n1[k];
    const double* bk = k == 0 ? b0 : hw + H.off[k];
    double* xk = k == 0 ? x0 : hw + H.off[k] + (int64_t)n1 * n1;
    if (down) {
      if (k == last) {
        for (int i = threadIdx.x; i < n1 * n1; i += NT) xk[i] = bk[i];
        __syncthreads();
        fdm_solve<NT>(n1, H.Vc, L.htl, L.htd, xk, rt);
        if (k == 0) break;
        --k;
        down = false;
        continue;
      }
      hmg_gs<NT>(H.band[k], n1, c, bk, xk, true);
      const int n1c = H.n1[k + 1];
      hmg_restrict<NT>(H.band[k], n1, c, bk, xk, rt, n1c, hw + H.off[k + 1], hw + H.off[k + 1] + (int64_t)n1c * n1c);
      once &= ~(1u << k);
      ++k;
      continue;
    }
    // back on level k from one W(k + 1)
    if (k + 1 < last && !(once & (1u << k))) {
      once |= 1u << k;
      ++k;
      down = true;
      continue;
    }
    const int n1c = H.n1[k + 1];
    hmg_prolong<NT>(n1, n1c, hw + H.off[k + 1] + (int64_t)n1c * n1c, xk);
    hmg_gs<NT>(H.band[k], n1, c, bk, xk, false);
    if (k == 0) break;
    --k;
  }
}

// one p-multigrid V-cycle from the zero guess on A d = r (Sec. 4, steps 1-5, in correction
// form: the outer FP64 loop supplies r = b - A x and adds d to x).
// Buffers: y (nin^2 doubles, LDS first), s (>= max(nin^2 VT, n1^2 doubles)), d (nin^2 VT).
template <typename VT, int MASK, int OCC, bool EXT>
__device__ void vcycle(const InstDev& I, const LevelDev& L, int nu1, int nu2, const VT* r, VT* d, VT* y, VT* s,
                       VT* sbuf, int ka, int zidx, VT* win, int zwin, int coarse, double* hw, double* stage,
                       Stg bst) {
  constexpr bool YL = MASK & kY;
  constexpr int NT = Build<OCC>::NT;
  constexpr bool ST = Staged<MASK, OCC>::value;
  // s = r - A_l d, staged through LDS when the vectors are in global memory
  auto resid = [&]() {
    if constexpr (!ST)
      apply_A<NT, VT, OCC>(I, L, d, r, s, y);
    else
      apply_A_st<NT, VT>(I, L, d, r, s, y, bst);
  };
  const int n = I.ndof;
  // the 1024-thread build reads the factors' slot tables laid out for 8 lanes per row
  const TriDev& TL = Build<OCC>::TG == 8 ? L.L8 : L.L;
  const TriDev& TU = Build<OCC>::TG == 8 ? L.U8 : L.U;
  // step 1: pre-smoothing d = S r, then nu1 - 1 further steps d += S (r - A d)
  trsv<VT, YL, true, OCC>(TL, ka, zidx, r, y, sbuf, win, zwin, bst);
  trsv<VT, YL, !YL, OCC>(TU, ka, zidx, y, y, sbuf, win, zwin, bst);
  for (int i = threadIdx.x; i < n; i += NT) d[i] = y[i];
  __syncthreads();
  for (int m = 1; m < nu1; ++m) {
    resid();
    trsv<VT, YL, !(MASK & kS), OCC>(TL, ka, zidx, s, y, sbuf, win, zwin, bst);
    trsv<VT, YL, !YL, OCC>(TU, ka, zidx, y, y, sbuf, win, zwin, bst);
    for (int i = threadIdx.x; i < n; i += NT) d[i] += y[i];
    __syncthreads();
  }
  // step 2: residual restricted to p = 1, r1 = (M1^L)^{-1} P^T (r - A d); r1 lands in s
  resid();
  double* c1 = (double*)s;
  double* c2 = (double*)y;
  if constexpr (!ST) {
    pass_x<NT, VT>(I.nin, I.nin, I.PxT, s, y);  // nin rows x n1 columns
    __syncthreads();
    pass_y<NT, VT>(I.n1, I.nin, I.PyT, y, (VT)1, (const VT*)nullptr, (VT)0, false, I.il1_y, I.il1_x, c1);
  } else {
    pass_x_st<NT, VT>(I.nin, I.nin, I.PxT, s, y, bst);
    __syncthreads();
    pass_y_st<NT, VT>(I.n1, I.nin, I.PyT, y, (VT)1, (const VT*)nullptr, (VT)0, false, I.il1_y, I.il1_x, c1, bst);
  }
  __syncthreads();
  // step 3: p = 1 solve (FP64), exact or by one h-multigrid W-cycle
  if (EXT && coarse == 1) {
    hmg_wcycle<NT>(I, L, c1, c2, hw);
    for (int i = threadIdx.x; i < I.ndof1; i += NT) c1[i] = c2[i];
    __syncthreads();
  } else {
    coarse_solve<NT, Build<OCC>::GBC>(I, L, c1, c2, stage);
    // the staging area may overlap the triangular solves' window: restore its zero word, which the
    // solves read for padding entries (FP64 data left there can read as a NaN in FP32)
    if (stage && win && threadIdx.x == 0) win[zwin] = (VT)0;
  }
  // step 4: prolongation and update d += (Mp^L)^{-1} P e1
  if constexpr (!ST) {
    pass_x<NT, VT>(I.n1, I.n1, I.Px, c1, y);  // n1 rows x nin columns
    __syncthreads();
    pass_y<NT, VT>(I.nin, I.n1, I.Py, y, (VT)1, (const VT*)nullptr, (VT)0, true, I.ilp_y, I.ilp_x, d);
  } else {
    pass_x_st<NT, VT>(I.n1, I.n1, I.Px, c1, y, bst);
    __syncthreads();
    pass_y_st<NT, VT>(I.nin, I.n1, I.Py, y, (VT)1, (const VT*)nullptr, (VT)0, true, I.ilp_y, I.ilp_x, d, bst);
  }
  __syncthreads();
  // step 5: nu2 post-smoothing steps d += S (r - A d)
  for (int m = 0; m < nu2; ++m) {
    resid();
    trsv<VT, YL, !(MASK & kS), OCC>(TL, ka, zidx, s, y, sbuf, win, zwin, bst);
    trsv<VT, YL, !YL, OCC>(TU, ka, zidx, y, y, sbuf, win, zwin, bst);
    for (int i = threadIdx.x; i < n; i += NT) d[i] += y[i];
    __syncthreads();
  }
}

// Conjugate gradients preconditioned by diag(A_l) (the comparison solver of Sec. 4 and Sec. 5),
// FP64, textbook recursion from the iterate in x until ||r|| <= tol ||b|| (r updated by the
// recursion) or maxcyc iterations.  r, p, q, tmp: work vectors of n_dof doubles.  Returns the
// iterations; sets status bit 0 (non-finite) or 1 (cap).
template <int NT, int OCC>
__device__ __forceinline__ int pcg(const InstDev& I, const LevelDev& L, const double* b, double* x, double* r, double* p, double* q,
                   double* tmp, double* red, double stol2, double bn2, int maxcyc, int* status) {
  const int n = I.ndof;
  const G<double>* __restrict__ dg = gp(L.dgA);
  double rn2 = block_sum<NT>(apply_A<NT, double, OCC>(I, L, x, b, r, tmp), red);  // r = b - A x
  double rho_old = 0.0;
  int it = 0;
  for (;; ++it) {
    if (!(rn2 <= 1.0e300)) {
      if (threadIdx.x == 0) atomicOr(status, 1);
      break;
    }
    if (rn2 <= stol2 * bn2) break;
    if (it >= maxcyc) {
      if (threadIdx.x == 0) atomicOr(status, 2);
      break;
    }
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) part += r[i] * (r[i] / dg[i]);
    const double rho = block_sum<NT>(part, red);  // r . z with z = D^{-1} r
    if (it == 0) {
      for (int i = threadIdx.x; i < n; i += NT) p[i] = r[i] / dg[i];
    } else {
      const double beta = rho / rho_old;
      for (int i = threadIdx.x; i < n; i += NT) p[i] = r[i] / dg[i] + beta * p[i];
    }
    __syncthreads();
    apply_A<NT, double, OCC>(I, L, p, (const double*)nullptr, q, tmp);  // q = -A p
    part = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) part += p[i] * q[i];
    const double alpha = -rho / block_sum<NT>(part, red);
    part = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
      x[i] += alpha * p[i];
      r[i] += alpha * q[i];
      part += r[i] * r[i];
    }
    rn2 = block_sum<NT>(part, red);
    rho_old = rho;
  }
  return it;
}

template <typename VT, int MASK, int OCC, bool EXT = false>
__device__ __forceinline__ void phi_body(const PhiParams& P, const LdsPlan& plan) {
  constexpr int NT = Build<OCC>::NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const PhiJob job = P.jobs[blockIdx.x];
  // an instance whose MGRIT residual has reached the tolerance is left as it is
  if (P.frozen && P.frozen[job.inst]) return;
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

  // the triangular solves read padding columns from the LDS word y[zidx], which stays zero, and
  // read sbuf (kSbufWords words) beyond a level's rows with zero coefficients: make it finite once
  if ((MASK & kY) && threadIdx.x == 0) y[plan.zidx] = (VT)0;
  // window of the triangular solves when y is in global memory; its zero word likewise
  VT* win = (!(MASK & kY) && plan.off_win >= 0) ? (VT*)(smem + plan.off_win) : nullptr;
  // LDS staging area of the p = 1 transforms (it may share the window's bytes: the two are never in
  // use at once)
  double* stage = plan.off_stage >= 0 ? (double*)(smem + plan.off_stage) : nullptr;
  if (win && threadIdx.x == 0) win[plan.zwin] = (VT)0;
  // LDS staging area of the band passes when y is in global memory
  Stg bst;
  if constexpr (Staged<MASK, OCC>::value) {
    if (plan.off_bst >= 0) {
      bst.p = smem + plan.off_bst;
      bst.bytes = plan.bst_bytes;
    }
  }
  for (int i = threadIdx.x; i < kSbufWords; i += NT) sbuf[i] = (VT)0;
  double* Vl = P.vtab ? P.vtab[job.inst * kMaxLevels + job.level] : nullptr;
  const double* Gl = (P.gtab && job.level > 0) ? P.gtab[job.inst * kMaxLevels + job.level] : nullptr;
  const double* Fv = I.F;
  const double* scale = I.scale;
  const double stol2 = job.level == 0 ? P.stol * P.stol : P.stolc * P.stolc;
  int total = 0;
  for (int st = 0; st < job.len; ++st) {
    const int k = job.k0 + P.kshift + st;  // step from point k to point k + 1
    const double* g1 = Gl ? Gl + (int64_t)(k + 1) * n : nullptr;
    double* tgt = Vl ? Vl + (int64_t)(k + 1) * n : nullptr;
    // right-hand side b = M v_k + dt f_{k+1} (level 0) or M v_k, and the initial iterate
    if (P.mode == kModeGiven) {
      const double* bg = P.bgiven + (int64_t)blockIdx.x * n;
      const double* xg = P.xgiven + (int64_t)blockIdx.x * n;
      for (int i = threadIdx.x; i < n; i += NT) {
        b[i] = bg[i];
        x[i] = xg[i];
      }
    } else {
      const double* vk = Vl + (int64_t)k * n;
      const double c = job.level == 0 ? scale[k + 1] : 0.0;
      if ((!EXT || L.cb == 0.0) && Staged<MASK, OCC>::value) {  // implicit Euler, staged passes
        pass_x_st<NT, double>(I.nin, I.nin, I.Mx, vk, yd, bst);
        __syncthreads();
        pass_y_st<NT, double>(I.nin, I.nin, I.My, yd, 1.0, job.level == 0 ? Fv : (const double*)nullptr, c, false,
                              nullptr, nullptr, b, bst);
      } else if (!EXT || L.cb == 0.0) {  // implicit Euler: B_l = M
        pass_x<NT, double>(I.nin, I.nin, I.Mx, vk, yd);
        __syncthreads();
        pass_y<NT, double>(I.nin, I.nin, I.My, yd, 1.0, job.level == 0 ? Fv : (const double*)nullptr, c, false,
                           nullptr, nullptr, b);
      } else {  // theta < 1: B_l = My (x) (Mx - cb Kx) - cb Ky (x) Mx2
        pass_x<NT, double>(I.nin, I.nin, L.XB, vk, yd);
        __syncthreads();
        pass_y<NT, double>(I.nin, I.nin, I.My, yd, 1.0, job.level == 0 ? Fv : (const double*)nullptr, c, false,
                           nullptr, nullptr, b);
        __syncthreads();
        pass_x<NT, double>(I.nin, I.nin, I.Mx2, vk, yd);
        __syncthreads();
        pass_y<NT, double>(I.nin, I.nin, I.Ky, yd, -L.cb, (const double*)nullptr, 0.0, true, nullptr, nullptr, b);
      }
      // initial iterate: 0 zero; 1 previous point; 2 current target at level 0 (the previous
      // MGRIT iterate), previous point at coarse levels (their state restarts from zero);
      // 4 at level 0: the current target (there a prediction) or the previous point, whichever
      // leaves the smaller residual
      const bool prev = P.guess == 1 || (P.guess >= 2 && job.level > 0);
      for (int i = threadIdx.x; i < n; i += NT) x[i] = prev ? vk[i] : (P.guess >= 2 ? tgt[i] : 0.0);
      if (P.guess == 4 && job.level == 0 && !(job.flags & 1)) {
        __syncthreads();
        double* rt = sizeof(VT) == 8 ? (double*)r : (double*)(ws + 5 * nm);  // FP64 residual temp
        const double ra = block_sum<NT>(apply_A<NT, double, OCC>(I, L, x, b, rt, yd), red);
        const double rp = block_sum<NT>(apply_A<NT, double, OCC>(I, L, vk, b, rt, yd), red);
        if (!(ra <= rp))
          for (int i = threadIdx.x; i < n; i += NT) x[i] = vk[i];
      }
    }
    __syncthreads();
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) part += b[i] * b[i];
    const double bn2 = block_sum<NT>(part, red);
    int cyc = 0;
    if (bn2 == 0.0) {  // zero right-hand side: the solution is exactly zero
      for (int i = threadIdx.x; i < n; i += NT) x[i] = 0.0;
      __syncthreads();
    }
    bool cg = false;
    if constexpr (EXT && sizeof(VT) == 8) {
      if (P.solver == 1) {
        cg = true;
        if (bn2 != 0.0)
          cyc = pcg<NT, OCC>(I, L, b, x, (double*)r, (double*)d, (double*)s, yd, red, stol2, bn2, P.maxcyc, P.status);
      }
    }
    for (; bn2 != 0.0 && !cg;) {
      // FP64 residual r = b - A x (stored in the V-cycle precision) and its norm
      part = 0.0;
      // Fused form (one first- and one second-direction pass, written straight into r) where LDS
      // holds a second FP64 temporary of n values: the d and s slots (FP32, contiguous) or the
      // d slot (FP64), both free here.  Elsewhere the four-pass form, which rounds the same way.
      constexpr bool FUSE = sizeof(VT) == 8 ? (MASK & kD) != 0 : ((MASK & kD) && (MASK & kS));
      bool fused = false;
      if constexpr (FUSE) {
        if (fusable<NT>(I, L)) {
          double* t2 = (double*)(smem + plan.off_d);
          pass_x2<NT, double>(I.nin, I.nin, L.X1, I.Mx2, x, yd, t2);
          __syncthreads();
          part = pass_y2<NT, double>(I.nin, I.nin, I.My, I.Ky, yd, (const double*)t2, -1.0, -L.c, b, 1.0, r);
          __syncthreads();
          fused = true;
        }
      }
      if constexpr (Staged<MASK, OCC>::value) {
        // y in global memory: staged passes, fused through the d slot when it is in global memory
        // (free here), written straight into r
        if (!fused && bst.p && !(MASK & kD) && (sizeof(VT) == 8 || fusable<NT>(I, L))) {
          part = apply_A_st<NT, double>(I, L, x, b, r, yd, bst, ws + 4 * nm);
          fused = true;
        }
      }
      if (!fused) {
        if constexpr (sizeof(VT) == 8) {
          part = apply_A<NT, double, OCC>(I, L, x, b, r, yd);
        } else {
          // residual in FP64 through the FP64 temp, then rounded into r
          double* rr = (double*)(ws + 5 * nm);  // FP64 residual staging in global scratch
          part = apply_A<NT, double, OCC>(I, L, x, b, rr, yd);
          for (int i = threadIdx.x; i < n; i += NT) r[i] = (VT)rr[i];
        }
      }
      const double rn2 = block_sum<NT>(part, red);
      if (!(rn2 <= 1.0e300)) {  // NaN or Inf
        if (threadIdx.x == 0) atomicOr(P.status, 1);
        break;
      }
      if (rn2 <= stol2 * bn2) break;
      if (cyc >= P.maxcyc) {
        if (threadIdx.x == 0) atomicOr(P.status, 2);
        break;
      }
      vcycle<VT, MASK, OCC, EXT>(I, L, P.nu1, P.nu2, r, d, y, s, sbuf, plan.ka, plan.zidx, win, plan.zwin, P.coarse,
                                 ws + P.hmg_off, stage, bst);
      for (int i = threadIdx.x; i < n; i += NT) x[i] += (double)d[i];
      __syncthreads();
      ++cyc;
    }
    total += cyc;
    // output
    if (P.mode == kModeChain) {
      for (int i = threadIdx.x; i < n; i += NT) tgt[i] = x[i] + (g1 ? g1[i] : 0.0);
    } else if (P.mode == kModeResidual) {
      double* ro = P.gtab[job.inst * kMaxLevels + job.level + 1] + (int64_t)job.outj * n;
      part = 0.0;
      for (int i = threadIdx.x; i < n; i += NT) {
        double v = x[i] + (g1 ? g1[i] : 0.0) - tgt[i];
        ro[i] = v;
        part += v * v;
      }
      const double r2 = block_sum<NT>(part, red);
      if (threadIdx.x == 0) P.nrm2[blockIdx.x] = r2;
    } else {
      double* xg = P.xgiven + (int64_t)blockIdx.x * n;
      for (int i = threadIdx.x; i < n; i += NT) xg[i] = x[i];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    P.vcount[blockIdx.x] += total;
    if (P.vlast) P.vlast[blockIdx.x] = total;
    if (total) atomicAdd(P.vinst + job.inst, (unsigned long long)total);
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
                               int ncoarse, const int* __restrict__ frozen) {
  if (frozen && *frozen) return;  // the instance has converged: its iterate stays as it is
  const int64_t tot = (int64_t)ncoarse * ndof;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / ndof + 1, i = t - (j - 1) * ndof;
    Vl[j * m * (int64_t)ndof + i] += Vc[j * (int64_t)ndof + i];
  }
}

// per instance: sum of the residual norms of its workgroups [begin[i], begin[i+1])
// ||r||^2 per instance from the per-workgroup partial sums of one group: workgroups
// begin[i] .. begin[i+1]-1 belong to the group's i-th instance, whose global id is id[i]
__global__ void norm_reduce_kernel(const double* __restrict__ nrm2, const int* __restrict__ begin,
                                   const int* __restrict__ id, double* __restrict__ out) {
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
    out[id[i]] = t;
  }
}

// ------------------------------------------------------------------------------------------
// host-side launch helpers (called from the driver)
// ------------------------------------------------------------------------------------------

// one workgroup per job; phi_kernel_o2 is the same code limited to 128 VGPRs per lane, so that
// two workgroups fit a CU when the LDS plan leaves room for them
template <typename VT, int MASK>
__global__ void __launch_bounds__(512) phi_kernel(PhiParams P, LdsPlan plan) {
  phi_body<VT, MASK, 1>(P, plan);
}
template <typename VT, int MASK>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) phi_kernel_o2(PhiParams P,
                                                                                          LdsPlan plan) {
  phi_body<VT, MASK, 2>(P, plan);
}
// the 1024-thread build (placement flag kT1024)
template <typename VT, int MASK>
__global__ void __launch_bounds__(1024) phi_kernel_t(PhiParams P, LdsPlan plan) {
  phi_body<VT, MASK, 3>(P, plan);
}
// the 512-thread build with 8 lanes per triangular-solve row (placement flag kW8)
template <typename VT, int MASK>
__global__ void __launch_bounds__(512) phi_kernel_w8(PhiParams P, LdsPlan plan) {
  phi_body<VT, MASK, 4>(P, plan);
}

// the extended build (512 threads, 4 lanes per row): also theta < 1 right-hand sides, the
// h-multigrid p = 1 solve and (FP64) the CG spatial solver; kept apart so that the other builds'
// register allocation carries none of that code
template <typename VT, int MASK>
__global__ void __launch_bounds__(512) phi_kernel_x(PhiParams P, LdsPlan plan) {
  phi_body<VT, MASK, 1, true>(P, plan);
}

using PhiFn = void (*)(PhiParams, LdsPlan);

template <typename VT>
static PhiFn pick(int mask) {
  if (mask & kExt) {
    switch (mask & 15) {
      case 15: return phi_kernel_x<VT, 15>;
      case 7: return phi_kernel_x<VT, 7>;
      case 3: return phi_kernel_x<VT, 3>;
      case 1: return phi_kernel_x<VT, 1>;
      default: return phi_kernel_x<VT, 0>;
    }
  }
  if (mask & kT1024) {
    switch (mask & 15) {
      case 15: return phi_kernel_t<VT, 15>;
      case 7: return phi_kernel_t<VT, 7>;
      case 3: return phi_kernel_t<VT, 3>;
      default: return phi_kernel_t<VT, 1>;
    }
  }
  if (mask & kW8) {
    switch (mask & 15) {
      case 15: return phi_kernel_w8<VT, 15>;
      case 7: return phi_kernel_w8<VT, 7>;
      case 3: return phi_kernel_w8<VT, 3>;
      default: return phi_kernel_w8<VT, 1>;
    }
  }
  if constexpr (sizeof(VT) == 4) {
    if (mask == (3 | kOcc2)) return phi_kernel_o2<VT, 3>;
    if (mask == (1 | kOcc2)) return phi_kernel_o2<VT, 1>;
    if (mask == kOcc2) return phi_kernel_o2<VT, 0>;  // window mode, two workgroups per CU
  }
  switch (mask & 15) {
    case 15: return phi_kernel<VT, 15>;
    case 7: return phi_kernel<VT, 7>;
    case 3: return phi_kernel<VT, 3>;
    case 1: return phi_kernel<VT, 1>;
    default: return phi_kernel<VT, 0>;
  }
}

// ------------------------------------------------------------------------------------------
// fixed device scratch of the allocation-free spatial-solve entry point
// ------------------------------------------------------------------------------------------
// kScratchDoubles doubles (64 MiB) per device, held until the process ends.  Host code must not use
// the array's name as a device address: scratch_setup resolves the address once per device (with that
// device current) and keeps it.
static __device__ __align__(256) double scratch[kScratchDoubles];

static double* g_scratch_ptr[kMaxDevices] = {};
static int g_scratch_ready[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// call with `device` current
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ready[device]) return hipSuccess;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (double*)ptr;
  g_scratch_ready[device] = 1;
  return hipSuccess;
}

double* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices && g_scratch_ready[device]) ? g_scratch_ptr[device] : nullptr;
}

// allow the kernel of a placement the device's whole per-workgroup LDS: several plans (wide and
// narrow placements, launch groups, autotuner probes) may share one kernel, and each launch
// requests its own plan's size (occupancy follows the launch's request, not this limit)
hipError_t phi_prepare(int fp32, int mask, int lds_bytes) {
  PhiFn f = fp32 ? pick<float>(mask) : pick<double>(mask);
  int dev = 0, mx = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  if (lds_bytes > mx) return hipErrorInvalidValue;
  return hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
}

hipError_t phi_launch(int fp32, int mask, int lds_bytes, const PhiParams& P, const LdsPlan& plan, int nblocks,
                      hipStream_t st) {
  PhiFn f = fp32 ? pick<float>(mask) : pick<double>(mask);
  hipLaunchKernelGGL(f, dim3(nblocks), dim3(mask & kT1024 ? 1024 : 512), lds_bytes, st, P, plan);
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

hipError_t correct_launch(double* Vl, const double* Vc, int ndof, int m, int ncoarse, const int* frozen,
                          hipStream_t st) {
  int64_t tot = (int64_t)ncoarse * ndof;
  if (tot <= 0) return hipSuccess;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(correct_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Vl, Vc, ndof, m, ncoarse, frozen);
  return hipGetLastError();
}

hipError_t norm_reduce_launch(const double* nrm2, const int* begin, const int* id, double* out, int ninst,
                              hipStream_t st) {
  hipLaunchKernelGGL(norm_reduce_kernel, dim3(ninst), dim3(256), 0, st, nrm2, begin, id, out);
  return hipGetLastError();
}

}  // namespace pmg
