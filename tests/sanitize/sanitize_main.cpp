// Host code under AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure only): the plan builders of both solvers for every
// distance, the FP64 oracle's procedures on small codes, and the sweep
// kernels' own source on the host emulation (one work-group of host threads)
// for a forward and an adjoint at d = 3 and a truncated forward at d = 5.
// Exit status 0 and no sanitizer report = clean.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "emu_hip.hpp"

#include "adjoint.hpp"
#include "kw_plan.hpp"

extern "C" {
int orc_transfer(int d, const double* rates, int nmodels, const int32_t* model_index, const uint8_t* syn, int64_t count,
                 double* logz, int threads);
int orc_enumerate(int d, const double* rates, double* table, double* marg);
int orc_rbim(int d, double p, const uint8_t* syn, double* logZ);
int orc_grad_logp(int d, const double* rates, const uint8_t* syn, double* grad, double* logp);
}

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

int fails = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++fails;
  }
}

// forward of one syndrome on the emulated work-group, exact plan (chi = 0) or truncated
template <typename Real, typename Fac>
void emu_forward(int d, int chi, int group, const std::vector<double>& rates, const std::vector<uint8_t>& syn,
                 double* logz, unsigned* status) {
  Plan p;
  expect(build_plan(d, chi, group, &p).empty(), "build_plan");
  const LdsLayout lay = lds_layout(p.h, sizeof(Real), sizeof(Fac));
  std::vector<uint8_t> smem(lay.bytes + 64);
  std::vector<Real> scr(p.h.scratch_elems + 64), snap(p.h.mps_elems + 64);
  JobDev job{p.blob.data(), rates.data(), nullptr, syn.data(), logz, nullptr, nullptr, 1, 0, 0, 1, 0, status};
  Barriers bars;
  run_block([&](int) { contract_syndrome<Real, Fac>(job, 0, smem.data(), lay, scr.data(), snap.data()); });
}

}  // namespace

int main() {
  // plan builders, every distance, and the LDS carve-up
  for (int d = 3; d <= 31; d += 2) {
    for (int chi : {0, 4, 16, 32}) {
      if (chi == 0 && d > 7) continue;
      for (int g = 1; g <= 2; ++g) {
        Plan p;
        const std::string e = build_plan(d, chi, g, &p);
        if (!e.empty()) continue;  // refused shapes are an answer, not an error
        for (int aj = 0; aj < 2; ++aj) {
          const LdsLayout l = lds_layout(p.h, 4, 8, aj != 0);
          expect(l.bytes > 0, "lds_layout");
        }
        PlanHeader acc{};
        merge_maxima(&acc, p.h);
      }
    }
    KwPlan kp;
    expect(build_kw_plan(d, &kp).empty(), "build_kw_plan");
    expect(kp.h.N == 2 * (d * d + 1), "kw order");
  }
  // oracle procedures
  {
    const int d = 3, n = 9, m = 8;
    std::vector<double> rates(n * 3, 0.04), table(256 * 4), marg(256 * n * 4), logz(4), grad(n * 3);
    expect(orc_enumerate(d, rates.data(), table.data(), marg.data()) >= 0, "orc_enumerate");
    std::vector<uint8_t> syn(m, 0);
    syn[1] = 1;
    expect(orc_transfer(d, rates.data(), 1, nullptr, syn.data(), 1, logz.data(), 1) >= 0, "orc_transfer");
    double lp = 0;
    expect(orc_grad_logp(d, rates.data(), syn.data(), grad.data(), &lp) >= 0, "orc_grad_logp");
    expect(orc_rbim(d, 0.1, syn.data(), logz.data()) >= 0, "orc_rbim");
    std::vector<double> r5(25 * 3, 0.03), lz5(4);
    std::vector<uint8_t> s5(24, 0);
    s5[3] = s5[7] = 1;
    expect(orc_transfer(5, r5.data(), 1, nullptr, s5.data(), 1, lz5.data(), 1) >= 0, "orc_transfer d=5");
  }
  // kernel source on the host emulation
  {
    const int d = 3, n = 9, m = 8;
    std::vector<double> rates(n * 3);
    for (int i = 0; i < n * 3; ++i) rates[i] = 0.01 + 0.003 * i;
    std::vector<uint8_t> syn(m, 0);
    syn[2] = syn[5] = 1;
    double lz[4], ref[4];
    unsigned st[4] = {0, 0, 0, 0};
    emu_forward<double, double>(d, 0, 2, rates, syn, lz, st);
    expect(orc_transfer(d, rates.data(), 1, nullptr, syn.data(), 1, ref, 1) >= 0, "oracle ref");
    for (int k = 0; k < 4; ++k) expect(std::fabs(lz[k] - ref[k]) < 1e-10 * (1 + std::fabs(ref[k])), "emu forward d=3");
    emu_forward<float, float>(d, 2, 1, rates, syn, lz, st);  // truncated, FP32
    // adjoint
    Plan p;
    build_plan(d, 0, 2, &p);
    const LdsLayout lay = lds_layout(p.h, 8, 8);
    const int S = p.h.shared_rows < p.h.nstep ? p.h.shared_rows : p.h.nstep;
    const int64_t elems = 2 * p.h.scratch_elems + (int64_t)(S + 4 * (p.h.nstep - S)) * p.h.mps_elems +
                          p.h.env_elems + 3 * p.h.tmp_elems;
    std::vector<uint8_t> smem(lay.bytes + 64);
    std::vector<double> scr(elems + 64), part(n * 3, 0.0);
    double logp = 0, gp = 1.0, lzb[4];
    JobDev job{p.blob.data(), rates.data(), nullptr, syn.data(), lzb, &logp, &gp, 1, 0, 0, 1, 0, st};
    Barriers bars;
    run_block([&](int) { adjoint_syndrome<double, double, GEMM_VALU>(job, 0, smem.data(), lay, scr.data(), 1, part.data()); });
    double g[27], lpr = 0;
    orc_grad_logp(d, rates.data(), syn.data(), g, &lpr);
    for (int i = 0; i < n * 3; ++i) expect(std::fabs(part[i] - g[i]) < 1e-9 * (1 + std::fabs(g[i])), "emu adjoint d=3");
    // truncated d = 5 forward
    std::vector<double> r5(25 * 3, 0.02);
    std::vector<uint8_t> s5(24, 0);
    s5[4] = 1;
    emu_forward<double, double>(5, 4, 2, r5, s5, lz, st);
  }
  std::printf("sanitized host run: %d failures\n", fails);
  return fails ? 1 : 0;
}
