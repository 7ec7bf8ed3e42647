// The chunk schedule of a transport round, on the CPU: the home workgroups
// of ctd_schedule.h and the claim protocol the kernel follows with them.
// Reads "seed grid waves n_0 ... n_{k-1}" lines (chunks per case) from stdin;
// for each, plays the protocol with a pseudo-random interleaving of the
// waves and prints "ok" or the first violation.  Protocol: workgroup g starts
// on the last case whose home workgroups start at or before g; a wave's
// first claim in its home case is its rank (g - wg_lo) * waves + w, every
// other claim of case c is home_waves[c] + (counter c)++; a claim at or past
// the case's chunk count ends the wave's claims; when every wave of a
// workgroup has ended its claims and drained, the workgroup picks the next
// case, cyclically from c + 1, with home_waves + counter below its chunk
// count, or exits.  Every chunk must run exactly once and every workgroup
// must exit.
#include <cstdint>
#include <cstdio>
#include <sstream>
#include <string>
#include <vector>

#include "ctd_schedule.h"

namespace {

struct Rng {
  uint64_t s;
  uint32_t next() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(s >> 33);
  }
};

std::string play(uint64_t seed, int grid, int waves, const std::vector<uint64_t> &n) {
  const int nrc = (int)n.size();
  std::vector<uint64_t> begin((size_t)nrc), end((size_t)nrc);
  uint64_t t = 0;
  for (int i = 0; i < nrc; ++i) {
    begin[i] = t;
    t += n[i];
    end[i] = t;
  }
  std::vector<uint32_t> lo((size_t)nrc), hw((size_t)nrc);
  ctd::home_workgroups(begin.data(), nrc, grid, waves, lo.data(), hw.data());
  uint64_t sum = 0;
  for (uint32_t h : hw) sum += h;
  if (sum != (uint64_t)grid * (uint64_t)waves) return "home waves do not add up to the grid";
  std::vector<uint64_t> ctr((size_t)nrc, 0), runs(t, 0);
  struct Wave { bool first = true, done = false; int work = 0; };
  struct Wg { int c = 0; bool home = true, exited = false; std::vector<Wave> w; };
  std::vector<Wg> wg((size_t)grid);
  for (int g = 0; g < grid; ++g) {
    int c = 0;
    for (int i = 0; i < nrc; ++i)
      if (lo[i] <= (uint32_t)g) c = i;
    if (!(lo[c] <= (uint32_t)g && (uint32_t)g < (c + 1 < nrc ? lo[c + 1] : (uint32_t)grid)))
      return "workgroup outside its home range";
    wg[g].c = c;
    wg[g].w.assign((size_t)waves, Wave());
  }
  Rng rng{seed};
  int live = grid;
  for (uint64_t step = 0; live > 0; ++step) {
    if (step > 100000000ull) return "no progress";
    const int g = (int)(rng.next() % (uint32_t)grid);
    Wg &W = wg[g];
    if (W.exited) continue;
    std::vector<int> busy;
    for (int i = 0; i < waves; ++i)
      if (!(W.w[i].done && W.w[i].work == 0)) busy.push_back(i);
    if (busy.empty()) {   // the barrier: pick the next case
      int nxt = -1;
      for (int i = 1; i <= nrc && nxt < 0; ++i) {
        const int d = (W.c + i) % nrc;
        if (hw[d] + ctr[d] < n[d]) nxt = d;
      }
      if (nxt < 0) {
        W.exited = true;
        --live;
        continue;
      }
      W.c = nxt;
      W.home = false;
      W.w.assign((size_t)waves, Wave());
      continue;
    }
    const int wi = busy[rng.next() % busy.size()];
    Wave &v = W.w[wi];
    if (v.work > 0) {
      --v.work;
      continue;
    }
    const int c = W.c;
    uint64_t k;
    if (W.home && v.first) k = (uint64_t)(g - (int)lo[c]) * (uint64_t)waves + (uint64_t)wi;
    else k = hw[c] + ctr[c]++;
    v.first = false;
    if (k >= n[c]) {
      v.done = true;
    } else {
      runs[begin[c] + k] += 1;
      v.work = (int)(rng.next() % 4);
    }
  }
  for (uint64_t i = 0; i < t; ++i)
    if (runs[i] != 1) return "chunk " + std::to_string(i) + " ran " + std::to_string(runs[i]) + " times";
  return "ok";
}

}  // namespace

int main() {
  char line[1 << 16];
  while (std::fgets(line, sizeof line, stdin)) {
    std::istringstream in(line);
    uint64_t seed;
    int grid, waves;
    if (!(in >> seed >> grid >> waves)) continue;
    std::vector<uint64_t> n;
    uint64_t x;
    while (in >> x) n.push_back(x);
    std::printf("%s\n", play(seed, grid, waves, n).c_str());
  }
  return 0;
}
