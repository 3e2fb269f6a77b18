// Host check of the register-resident line FFT (csrc/fft_reg.hpp, the same
// template the kernels instantiate): every listed length and both signs
// against the O(N^2) DFT in long double, in FP64 and FP32.  Prints one line
// per length: N, then the largest relative error of the four cases.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <random>

#include "../../paper_1603_02732_amd/csrc/fft_reg.hpp"

using sgo::cplx;

template <typename T, int N, int S>
double check() {
  std::mt19937 g(N * 7 + S + 3);
  std::uniform_real_distribution<double> u(-1, 1);
  cplx<T> in[N], out[N];
  double re[N], im[N];
  for (int i = 0; i < N; ++i) {
    re[i] = u(g);
    im[i] = u(g);
    in[i] = {(T)re[i], (T)im[i]};
  }
  sgo::freg::fft<T, S, N>(in, out);
  double err = 0, mx = 0;
  for (int k = 0; k < N; ++k) {
    long double sr = 0, si = 0;
    for (int n = 0; n < N; ++n) {
      const long double a = S * 2.0L * 3.14159265358979323846264338327950288L *
                            (long double)((long)n * k % N) / N;
      sr += re[n] * cosl(a) - im[n] * sinl(a);
      si += re[n] * sinl(a) + im[n] * cosl(a);
    }
    err = std::fmax(err, std::fabs((double)sr - (double)out[k].x));
    err = std::fmax(err, std::fabs((double)si - (double)out[k].y));
    mx = std::fmax(mx, std::fabs((double)sr));
  }
  return err / mx;
}

template <int N>
void line() {
  std::printf("%d %.3e %.3e %.3e %.3e\n", N, check<double, N, 1>(), check<double, N, -1>(),
              check<float, N, 1>(), check<float, N, -1>());
}

int main() {
  line<8>();
  line<12>();
  line<15>();
  line<27>();
  line<48>();
  line<50>();
  line<60>();
  line<64>();
  return 0;
}
