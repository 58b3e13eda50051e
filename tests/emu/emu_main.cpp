// Host entry points that run the device code of the sweep on NT host threads:
// the forward one syndrome (four cosets) at a time, the adjoint one
// (syndrome, coset) item at a time.  Test
// infrastructure only: built by tests/test_kernel_emulation.py.
#include "emu_hip.hpp"

#include "adjoint.hpp"

#include <cmath>
#include <cstdio>
#include <vector>

using namespace tnmld;

namespace {

struct Barriers {
  std::barrier<> block{NT};
  std::vector<std::barrier<>*> own;
  Barriers() {
    g_block_bar = &block;
    for (int w = 0; w < NT / 64; ++w) own.push_back(g_wave_bar[w] = new std::barrier<>(64));
    for (int r = 0; r < NT / 16; ++r) own.push_back(g_row_bar[r] = new std::barrier<>(16));
  }
  ~Barriers() {
    for (auto* b : own) delete b;
  }
};

template <class F>
void run_block(F f) {
  std::vector<std::thread> th;
  for (int t = 0; t < NT; ++t)
    th.emplace_back([&, t] {
      threadIdx.x = t;
      f(t);
    });
  for (auto& x : th) x.join();
}

template <typename Real, typename Fac>
int forward(int d, int chi, int group, const double* rates, int n_models, const int32_t* model_index,
            const uint8_t* syn, int count, double* logz, unsigned* status, int rounds = 1,
            const double* meas = nullptr, bool xg = false) {
  Plan p;
  if (!build_plan(d, chi, group, &p, rounds).empty()) return -1;
  // xg: the layout of the 256-thread launches that keep the LQ matrix of the
  // right-to-left sweep in the work-group's scratch (after the site regions)
  LdsLayout lay = lds_layout(p.h, sizeof(Real), sizeof(Fac), false, xg);
  const int64_t sbytes = (p.h.scratch_elems * (int64_t)sizeof(Real) + 255) / 256 * 256;
  if (xg) lay.xg = (int32_t)sbytes;
  std::vector<double> smem(lay.bytes / 8 + 16), scr((sbytes + (int64_t)p.h.max_X * sizeof(Fac)) / 8 + 16),
      snap(p.h.mps_elems * sizeof(Real) / 8 + 16);
  JobDev job{p.blob.data(), rates, model_index, syn, logz, nullptr, nullptr, count, 0, 0, n_models, rounds, status,
             meas};
  Barriers bars;
  for (int b = 0; b < count; ++b)
    run_block([&](int) {
      if (xg)
        contract_syndrome<Real, Fac, GEMM_VALU, true>(job, b, (uint8_t*)smem.data(), lay, (Real*)scr.data(),
                                                      (Real*)snap.data());
      else
        contract_syndrome<Real, Fac>(job, b, (uint8_t*)smem.data(), lay, (Real*)scr.data(), (Real*)snap.data());
    });
  return 0;
}

template <typename Real, typename Fac>
int gradient(int d, int chi, int group, const double* rates, const uint8_t* syn, int count, const double* logz,
             const double* logp, const double* gradp, double* out) {
  Plan p;
  if (!build_plan(d, chi, group, &p).empty()) return -1;
  const PlanHeader& H = p.h;
  const LdsLayout lay = lds_layout(H, sizeof(Real), sizeof(Fac));
  const int S = H.shared_rows < H.nstep ? H.shared_rows : H.nstep;
  const int64_t elems = 2 * H.scratch_elems + (int64_t)(S + 4 * (H.nstep - S)) * H.mps_elems + H.env_elems +
                        3 * H.tmp_elems;
  std::vector<double> smem(lay.bytes / 8 + 16), scr(elems * sizeof(Real) / 8 + 16);
  JobDev job{p.blob.data(), rates, nullptr, syn, const_cast<double*>(logz), logp, gradp, count, 0, 0, 1, 0, nullptr};
  Barriers bars;
  for (int b = 0; b < count; ++b)
    run_block([&](int) {
      adjoint_syndrome<Real, Fac, GEMM_VALU>(job, b, (uint8_t*)smem.data(), lay, (Real*)scr.data(), 0, out);
    });
  return 0;
}

}  // namespace

// precision: 0 = FP64, 1 = FP32 state with FP64 factorisations, 3 = plain FP32
extern "C" int emu_forward(int d, int chi, int precision, int group, const double* rates, const uint8_t* syn,
                           int count, double* logz) {
  if (precision == 0) return forward<double, double>(d, chi, group, rates, 1, nullptr, syn, count, logz, nullptr);
  if (precision == 1) return forward<float, double>(d, chi, group, rates, 1, nullptr, syn, count, logz, nullptr);
  return forward<float, float>(d, chi, group, rates, 1, nullptr, syn, count, logz, nullptr);
}

// the same with the input site and the LQ matrix in global scratch (the
// staged explicit Q of the right-to-left sweep)
extern "C" int emu_forward_xg(int d, int chi, int precision, int group, const double* rates, const uint8_t* syn,
                              int count, double* logz) {
  if (precision == 0)
    return forward<double, double>(d, chi, group, rates, 1, nullptr, syn, count, logz, nullptr, 1, nullptr, true);
  if (precision == 1)
    return forward<float, double>(d, chi, group, rates, 1, nullptr, syn, count, logz, nullptr, 1, nullptr, true);
  return forward<float, float>(d, chi, group, rates, 1, nullptr, syn, count, logz, nullptr, 1, nullptr, true);
}

// the same with noise models selected per syndrome and the call's status word
extern "C" int emu_forward_models(int d, int chi, int precision, int group, const double* rates, int n_models,
                                  const int32_t* model_index, const uint8_t* syn, int count, double* logz,
                                  unsigned* status) {
  if (precision == 0)
    return forward<double, double>(d, chi, group, rates, n_models, model_index, syn, count, logz, status);
  if (precision == 1)
    return forward<float, double>(d, chi, group, rates, n_models, model_index, syn, count, logz, status);
  return forward<float, float>(d, chi, group, rates, n_models, model_index, syn, count, logz, status);
}

// repeated noisy rounds (group 1): syndromes [count][rounds][m], meas [m]
extern "C" int emu_forward_rounds(int d, int chi, int precision, int rounds, const double* rates, const double* meas,
                                  const uint8_t* syn, int count, double* logz, unsigned* status) {
  if (precision == 0)
    return forward<double, double>(d, chi, 1, rates, 1, nullptr, syn, count, logz, status, rounds, meas);
  if (precision == 1)
    return forward<float, double>(d, chi, 1, rates, 1, nullptr, syn, count, logz, status, rounds, meas);
  return forward<float, float>(d, chi, 1, rates, 1, nullptr, syn, count, logz, status, rounds, meas);
}

extern "C" int emu_gradient(int d, int chi, int precision, int group, const double* rates, const uint8_t* syn,
                            int count, const double* logz, const double* logp, const double* gradp, double* out) {
  if (precision == 0) return gradient<double, double>(d, chi, group, rates, syn, count, logz, logp, gradp, out);
  if (precision == 1) return gradient<float, double>(d, chi, group, rates, syn, count, logz, logp, gradp, out);
  return gradient<float, float>(d, chi, group, rates, syn, count, logz, logp, gradp, out);
}
