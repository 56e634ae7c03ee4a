// net.hpp -- learned warm start: a small convolutional network over the coefficient grid.
//
// Definition (not part of the paper; it supplies initial iterates for the implicit Euler solves):
// input planes u_k / s, (dt F / m) / s (m = row-sum-lumped mass) and ln(kappa dt n^2) / 4 on the
// (n+p) x (n+p) coefficient grid, s = rms(u_k) + rms(dt F / m); four 3x3 cross-correlations with
// zero padding, channels 3 -> 32 -> 32 -> 32 -> 1, ReLU after the first three; guess = u_k + s y.
// Parameters: one flat float array, per layer weights [cout][cin][3][3] then bias [cout].
//
// Arithmetic: BF16 weights, inputs and hidden activations (and hidden gradients in training),
// FP32 accumulation; the two 32 -> 32 layers (95 % of the work) run on the matrix cores
// (v_mfma_f32_16x16x32_bf16), the thin first and last layers on the vector ALUs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace pmg {

constexpr int kNetC = 32;  // hidden channels
constexpr int kNetParams = (32 * 3 * 9 + 32) + 2 * (32 * 32 * 9 + 32) + (1 * 32 * 9 + 1);

// one source of samples: a trajectory of (N_t + 1) rows of nin^2 FP64 coefficients and its data
struct NetSrc {
  const double* U;     // rows k = 0 .. N_t (row stride nin^2)
  double* Uout;        // where guesses are written (row k + 1), may equal U
  const double* F;     // load vector (nin^2)
  const double* ilx;   // 1 / lumped mass per direction (nin): 1 / m_i = ilx[ix] ily[iy]
  const double* ily;
  const double* scale; // source weight of step k -> k + 1 at entry k + 1 (null: dt)
  // K = My (x) Kx + Ky (x) Mx2 as interior band arrays, bw = 2p + 1 entries per row
  const double *My, *Ky, *Kx, *Mx2;
  double dt;           // step of the solves the guesses are for
  double kdt;          // kappa dt
  double lnc;          // ln(kappa dt n^2) / 4
  int nin, G, p, bw;
};

struct NetPick {
  int src, k;  // sample = (source, step k -> k + 1)
};

class NetState {
 public:
  ~NetState();
  hipError_t init(int device);
  hipError_t load(const float* theta_host);          // also resets the optimiser state
  hipError_t save(float* theta_host) const;
  hipError_t reserve(int nb, int G);                  // activation buffers for nb samples of grid G
  // raw network: x (nb x 3 x G x G float) -> y (nb x G x G float)
  hipError_t forward(int nb, int G, const float* x, float* y, hipStream_t st);
  // loss and gradient of a batch with targets t (nb x G x G); gradient stays on the device
  hipError_t backward(int nb, int G, const float* x, const float* t, hipStream_t st);
  hipError_t loss_and_grad(int nb, int G, const float* x, const float* t, float* grad_host, double* loss_host,
                           hipStream_t st);
  hipError_t adam_step(float lr, hipStream_t st);
  // samples from trajectories: planes (and targets when with_target) for picks[0..nb)
  hipError_t pack(const NetSrc* src_dev, const NetPick* pick_dev, int kbase, int nb, int G, bool with_target,
                  hipStream_t st);
  // guesses U_out[k + 1] = U[k] + s y for the packed samples
  hipError_t unpack(const NetSrc* src_dev, const NetPick* pick_dev, int kbase, int nb, int G, hipStream_t st);
  // predicted increments for the packed samples (pack, forward, unpack)
  hipError_t predict(const NetSrc* src_dev, const NetPick* pick_dev, int kbase, int nb, int G, hipStream_t st);
  // one training step on packed samples (pack with targets, forward, backward, Adam); loss on the device
  hipError_t train_packed(const NetSrc* src_dev, const NetPick* pick_dev, int nb, int G, float lr, hipStream_t st);
  hipError_t read_loss(double* loss_host, hipStream_t st);

  float* x_buf() { return x_; }
  float* t_buf() { return t_; }
  double* s_buf() { return s_; }

  bool loaded = false;
  int64_t steps = 0;
  double last_ms = 0;

 private:
  hipError_t run_forward(int nb, int G, const float* x, float* y, hipStream_t st);
  hipError_t run_backward(int nb, int G, const float* x, const float* t, hipStream_t st);
  hipError_t convert(hipStream_t st);
  hipError_t layout(int G, hipStream_t st);
  std::vector<void*> allocs_;
  template <class T>
  hipError_t alloc(T** p, size_t n);
  int device_ = -1;
  // parameters (flat FP32 master copy), Adam moments, gradient
  float *theta_ = nullptr, *m_ = nullptr, *v_ = nullptr, *grad_ = nullptr;
  // kernel layouts: layer 0 and 3 weights as BF16-rounded floats, layers 1 and 2 as BF16
  float *w0_ = nullptr, *w3_ = nullptr;
  uint16_t *wf1_ = nullptr, *wb1_ = nullptr, *wf2_ = nullptr, *wb2_ = nullptr;
  // activations (BF16, pixel-major with a zero halo ring), planes and scratch
  int nb_cap_ = 0, G_cap_ = 0, G_last_ = -1;
  uint16_t *a0_ = nullptr, *a1_ = nullptr, *a2_ = nullptr, *ga_ = nullptr, *gb_ = nullptr;
  float *x_ = nullptr, *t_ = nullptr, *y_ = nullptr, *dy_ = nullptr;
  double* s_ = nullptr;
  double* ebuf_ = nullptr;    // explicit increments of the packed samples (FP64, nb x G^2)
  double* epart_ = nullptr;   // their per-chunk sums of u^2 and e^2
  float* part_ = nullptr;     // weight-gradient partial sums
  double* lpart_ = nullptr;   // loss partial sums
  double* loss_ = nullptr;
  int64_t part_cap_ = 0;
  std::vector<void*> sized_;  // buffers freed on re-reserve
};

}  // namespace pmg
