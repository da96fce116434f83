// Host run of the library's pass sequences (the same work items the GPU
// schedules, bandops_driver.hpp / bandops_items.hpp) for the loss unit
// logdet Q - y^T Q^{-1} y + tr(Q^{-1} S), with and without the fused
// next-pass chunk maps, on an uneven batch of every compiled bandwidth.  Every work item
// runs on the CPU, one after another; the two schedules must agree.  Built by
// tests/test_host_pipeline.py, with the address and undefined-behaviour
// sanitizers on the host code and with the fusion limit raised to every
// compiled bandwidth (-DBO_KMAX_FUSED=12).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../paper_1902_10078_amd/csrc/bandops_steps.hpp"

using namespace bo;

namespace {

template <int K> struct HostRun {
  const Args &a;
  int64_t count;
  template <class Item> int go() {
    for (int64_t i = 0; i < count; ++i) Item::run(a, i);
    return 0;
  }
};

template <int K> int host_step(int st, const Args &a, int64_t count) {
  HostRun<K> r{a, count};
  return with_item<K, double>(st, r);
}

// Every compiled bandwidth.
constexpr int kKs[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12};

struct HostBE {
  bool range_on(int) const { return true; }
  int step(int st, int K, int, const Args &a, int64_t count) {
    switch (K) {
      case 0: return host_step<0>(st, a, count);
      case 1: return host_step<1>(st, a, count);
      case 2: return host_step<2>(st, a, count);
      case 3: return host_step<3>(st, a, count);
      case 4: return host_step<4>(st, a, count);
      case 5: return host_step<5>(st, a, count);
      case 6: return host_step<6>(st, a, count);
      case 7: return host_step<7>(st, a, count);
      case 8: return host_step<8>(st, a, count);
      case 9: return host_step<9>(st, a, count);
      case 10: return host_step<10>(st, a, count);
      case 11: return host_step<11>(st, a, count);
      case 12: return host_step<12>(st, a, count);
      default: return -4;
    }
  }
  int clear(const Args &a, int64_t count) {
    for (int64_t i = 0; i < count; ++i) ClearPart::run(a, i);
    return 0;
  }
  int finalize(const Args &a, int64_t count) {
    for (int64_t i = 0; i < count; ++i) Finalize::run(a, i);
    return 0;
  }
};

uint64_t g_state = 0x9E3779B97F4A7C15ull;
double urand() {   // splitmix64, uniform in [0, 1)
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}
double nrand() { return urand() + urand() + urand() - 1.5; }

struct Outputs {
  std::vector<double> L, Sig, Lbar, Qbar, z, ybar, parts;
  std::vector<int32_t> info;
};

// One loss-unit run over the batch; fused selects the schedule.
Outputs run(const std::vector<ProbIn> &probs, const std::vector<double> &Q, const std::vector<double> &y,
            const std::vector<double> &S, int64_t nrows, bool fused) {
  Sched s;
  if (!build_sched(probs.data(), (int)probs.size(), 96, 32, 8, s)) {
    std::fprintf(stderr, "bad schedule\n");
    std::exit(2);
  }
  // every problem's group size is a power of two with at most G = 8 groups
  // whose two serial lengths, gsize + ngroup, no other such size beats
  for (const ProbDesc &d : s.probs) {
    const int64_t ng = d.nchunk > 0 ? (d.nchunk + d.gsize - 1) / d.gsize : 0;
    bool ok = d.gsize >= 1 && d.gsize <= 8 && (d.gsize & (d.gsize - 1)) == 0 && d.ngroup == ng &&
              (d.ngroup <= 8 || d.gsize == 8);
    for (int32_t g = 1; g <= 8; g *= 2) {
      const int64_t n2 = (d.nchunk + g - 1) / g;
      if ((n2 <= 8 || g == 8) && g + n2 < d.gsize + d.ngroup) ok = false;
    }
    if (!ok) {
      std::fprintf(stderr, "group size %d for %d chunks (%d groups)\n", d.gsize, d.nchunk, d.ngroup);
      std::exit(2);
    }
  }
  std::vector<unsigned char> ws(s.bytes);
  std::memcpy(ws.data() + s.off_tables, s.table_blob.data(), s.table_blob.size());
  Outputs o;
  o.L.assign(Q.size(), 0.0);
  o.Sig.assign(Q.size(), 0.0);
  o.Lbar.assign(Q.size(), 0.0);
  o.Qbar.assign(Q.size(), 0.0);
  o.z.assign(nrows, 0.0);
  o.ybar.assign(nrows, 0.0);
  o.parts.assign(3 * probs.size(), 0.0);
  o.info.assign(probs.size(), -1);
  Args A{};
  bind_sched(s, ws.data(), false, A);
  A.Q = Q.data();
  A.y = y.data();
  A.Sb = S.data();
  A.L = o.L.data();
  A.z = o.z.data();
  A.x = o.ybar.data();
  A.S = o.Sig.data();
  A.Lb = o.Lbar.data();
  A.Qb = o.Qbar.data();
  A.parts = o.parts.data();
  A.info = o.info.data();
  HostBE be;
  if (pipe_gauss_loss(be, s, A, 0, fused) != 0) {
    std::fprintf(stderr, "pipeline failed\n");
    std::exit(2);
  }
  return o;
}

double rel(const std::vector<double> &a, const std::vector<double> &b) {
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    num = std::fmax(num, std::fabs(a[i] - b[i]));
    den = std::fmax(den, std::fabs(b[i]));
  }
  return den > 0.0 ? num / den : num;
}

}  // namespace

int main() {
  // uneven problems of every bandwidth, several chunks and groups each
  const int nk = (int)(sizeof(kKs) / sizeof(kKs[0]));
  const int nprob = 3 * nk;
  std::vector<ProbIn> probs;
  int64_t boff = 0, voff = 0;
  for (int p = 0; p < nprob; ++p) {
    const int k = kKs[p % nk];
    const int64_t n = 300 + 97 * p + (p % 3) * 31;
    probs.push_back(ProbIn{n, k, k + 1, boff, voff});
    boff += n * (k + 1);
    voff += n;
  }
  std::vector<double> Q(boff, 0.0), S(boff, 0.0), y(voff, 0.0);
  for (const ProbIn &p : probs) {
    const int w = p.k + 1;
    std::vector<double> L0(p.n * w, 0.0);
    for (int64_t j = 0; j < p.n; ++j)
      for (int d = 0; d <= p.k; ++d)
        if (j + d < p.n) L0[j * w + d] = d == 0 ? 1.0 + urand() : 0.3 * nrand();
    // Q = band(L0 L0^T): Q[i][j] = sum_m L0[i][m] L0[j][m], m <= j <= i
    for (int64_t j = 0; j < p.n; ++j)
      for (int d = 0; d <= p.k && j + d < p.n; ++d) {
        const int64_t i = j + d;
        double acc = 0.0;
        for (int64_t m = (i - p.k > 0 ? i - p.k : 0); m <= j; ++m) acc += L0[m * w + (i - m)] * L0[m * w + (j - m)];
        Q[p.boff + j * w + d] = acc;
        S[p.boff + j * w + d] = d == 0 ? 2.0 * w + urand() : nrand();
      }
    for (int64_t j = 0; j < p.n; ++j) y[p.voff + j] = nrand();
  }
  const Outputs a = run(probs, Q, y, S, voff, false);
  const Outputs b = run(probs, Q, y, S, voff, true);
  for (int p = 0; p < nprob; ++p)
    if (a.info[p] != 0 || b.info[p] != 0) {
      std::printf("FAIL info %d %d at problem %d\n", a.info[p], b.info[p], p);
      return 1;
    }
  const double e[] = {rel(b.L, a.L), rel(b.z, a.z), rel(b.Sig, a.Sig), rel(b.Lbar, a.Lbar),
                      rel(b.Qbar, a.Qbar), rel(b.ybar, a.ybar), rel(b.parts, a.parts)};
  const char *nm[] = {"L", "z", "Sig", "Lbar", "Qbar", "ybar", "parts"};
  int bad = 0;
  for (int i = 0; i < 7; ++i) {
    std::printf("%s %.3e\n", nm[i], e[i]);
    if (!(e[i] <= 1e-11)) bad = 1;
  }
  std::printf("KMAX_FUSED %d\n", KMAX_FUSED);
  std::printf(bad ? "FAIL\n" : "host pipeline ok\n");
  return bad;
}
