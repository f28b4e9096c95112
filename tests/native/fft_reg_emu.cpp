// CPU emulation of one workgroup of the register-resident FFT passes.
//
// Runs the host-callable pieces of fft_reg.h (pass A in registers, the LDS
// exchange, pass B and the output layout) for every thread of one 256-thread
// block, with the barrier between them implied by running the threads in
// order, and compares each column (or row) with a naive DFT in double.
// Forward and inverse, for the column shapes (L, C) and row shapes (L, P)
// the library instantiates.  Prints one line per shape and exits non-zero
// on the first relative error above 1e-5.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2510_05206_amd/csrc/fft_reg.h"

using pm::freg::RowShape;
using pm::freg::Shape;

static int g_fail = 0;

template <class S, bool INV>
static void emulate(const char* name, int n_lines) {
  const int L = S::L;
  // twiddle table exp(-2 pi i t / L) read with stride 1 (Lmax = L)
  std::vector<float2> tw(L);
  for (int t = 0; t < L; ++t) tw[t] = make_float2((float)std::cos(-2 * M_PI * t / L), (float)std::sin(-2 * M_PI * t / L));
  // input: n_lines lines of L complex values, seeded LCG
  std::vector<double> xr(n_lines * L), xi(n_lines * L);
  unsigned long long st = 0x9e3779b97f4a7c15ull ^ (unsigned long long)(L * 131 + n_lines);
  auto rnd = [&]() {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (double)((st >> 11) & ((1ull << 53) - 1)) / (double)(1ull << 53) - 0.5;
  };
  for (int i = 0; i < n_lines * L; ++i) {
    xr[i] = rnd();
    xi[i] = rnd();
  }
  std::vector<float2> lds(S::LDS);
  std::vector<std::vector<float2>> v(256, std::vector<float2>(S::E));
  // load (input layout) + pass A + LDS store, every thread
  for (int tid = 0; tid < 256; ++tid) {
    const int c = S::lane_c(tid), n1 = S::lane_n1(tid);
    for (int r = 0; r < S::E; ++r) {
      const int t = S::t_in(n1, r);
      v[tid][r] = make_float2((float)xr[c * L + t], (float)xi[c * L + t]);
    }
    pm::freg::pass_a<S, INV>(v[tid].data(), n1, tw.data(), 1);
    pm::freg::store_y<S>(v[tid].data(), lds.data(), n1, c);
  }
  // barrier; pass B
  for (int tid = 0; tid < 256; ++tid) pm::freg::pass_b<S, INV>(v[tid].data(), lds.data(), S::lane_n1(tid), S::lane_c(tid));
  // compare the output layout with the naive DFT
  double num = 0, den = 0;
  for (int tid = 0; tid < 256; ++tid) {
    const int c = S::lane_c(tid), n1 = S::lane_n1(tid);
    for (int r = 0; r < S::E; ++r) {
      const int k = S::t_out(n1, r);
      double sr = 0, si = 0;
      for (int t = 0; t < L; ++t) {
        const double ang = (INV ? 2.0 : -2.0) * M_PI * (double)((long long)k * t % L) / L;
        sr += xr[c * L + t] * std::cos(ang) - xi[c * L + t] * std::sin(ang);
        si += xr[c * L + t] * std::sin(ang) + xi[c * L + t] * std::cos(ang);
      }
      num += (v[tid][r].x - sr) * (v[tid][r].x - sr) + (v[tid][r].y - si) * (v[tid][r].y - si);
      den += sr * sr + si * si;
    }
  }
  // every output index of every line is produced exactly once
  std::vector<int> seen(n_lines * L, 0);
  for (int tid = 0; tid < 256; ++tid)
    for (int r = 0; r < S::E; ++r) seen[S::lane_c(tid) * L + S::t_out(S::lane_n1(tid), r)]++;
  int bad_cover = 0;
  for (int i = 0; i < n_lines * L; ++i) bad_cover += seen[i] != 1;
  const double rel = std::sqrt(num / den);
  std::printf("%s L=%d %s rel %.3e cover %s\n", name, L, INV ? "inv" : "fwd", rel, bad_cover ? "BAD" : "ok");
  if (!(rel < 1e-5) || bad_cover) g_fail = 1;
}

template <int L, int C>
static void col() {
  emulate<Shape<L, C>, false>("cols", C);
  emulate<Shape<L, C>, true>("cols", C);
}
template <int L, int P>
static void row() {
  emulate<RowShape<L, P>, false>("rows", 256 / P);
  emulate<RowShape<L, P>, true>("rows", 256 / P);
}

int main() {
  // the column shapes launch_cols instantiates (C = 256 / P columns per block)
  col<16, 64>();
  col<32, 64>();
  col<64, 32>();
  col<128, 32>();
  col<256, 16>();
  col<512, 16>();
  col<1024, 8>();
  // the row shapes fft_rows instantiates (complex length L = n / 2)
  row<2, 1>();
  row<4, 2>();
  row<8, 2>();
  row<16, 4>();
  row<32, 4>();
  row<64, 8>();
  row<128, 8>();
  row<256, 16>();
  row<512, 16>();
  return g_fail;
}
