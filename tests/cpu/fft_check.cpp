// CPU check of the register-level transforms in csrc/mra_fft.h, exactly as
// the kernels call them (lane mappings included).  Prints "ok" or the first
// failure and exits non-zero.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2011_05755_amd/csrc/mra_fft.h"

using cd = std::complex<double>;
static const double kPi = 3.14159265358979323846;

static int fails = 0;
static void check(bool ok, const char* what, double err) {
  if (!ok) {
    std::printf("FAIL %s err=%g\n", what, err);
    ++fails;
  }
}

static float2 tw256(int e) {  // exp(-2 pi i e / 256)
  double a = 2 * kPi * (e & 255) / 256.0;
  return make_float2((float)std::cos(a), (float)-std::sin(a));
}

template <int N, int SIGN, class F>
static void test_small(F fn, const char* name, std::mt19937& rng) {
  std::normal_distribution<double> nd;
  float2 v[N];
  cd ref[N], in[N];
  for (int i = 0; i < N; ++i) {
    in[i] = cd(nd(rng), nd(rng));
    v[i] = make_float2((float)in[i].real(), (float)in[i].imag());
  }
  for (int n = 0; n < N; ++n) {
    ref[n] = 0;
    for (int k = 0; k < N; ++k) ref[n] += in[k] * std::polar(1.0, SIGN * 2 * kPi * k * n / N);
  }
  fn(v);
  double err = 0;
  for (int n = 0; n < N; ++n) err = std::fmax(err, std::abs(cd(v[n].x, v[n].y) - ref[n]));
  check(err < 1e-5, name, err);
}

int main() {
  std::mt19937 rng(1);
  std::normal_distribution<double> nd;
  for (int rep = 0; rep < 20; ++rep) {
    test_small<8, -1>([](float2(&v)[8]) { mra::dft8<-1>(v); }, "dft8 fwd", rng);
    test_small<8, +1>([](float2(&v)[8]) { mra::dft8<+1>(v); }, "dft8 inv", rng);
    test_small<16, -1>([](float2(&v)[16]) { mra::dft16<-1>(v); }, "dft16 fwd", rng);
    test_small<16, +1>([](float2(&v)[16]) { mra::dft16<+1>(v); }, "dft16 inv", rng);
  }

  // ---- forward ring FFT with 8 lanes -------------------------------------
  for (int rep = 0; rep < 20; ++rep) {
    double p[256];
    for (double& x : p) x = nd(rng);
    float2 Y[8][16];
    for (int l = 0; l < 8; ++l) {
      float2 z[16];
      for (int n1 = 0; n1 < 16; ++n1) z[n1] = make_float2((float)p[16 * n1 + 2 * l], (float)p[16 * n1 + 2 * l + 1]);
      mra::dft16<-1>(z);
      for (int k1 = 0; k1 < 16; ++k1) Y[l][k1] = mra::cmul(z[k1], tw256(2 * ((l * k1) & 127)));
    }
    std::vector<int> seen(129, 0);
    double err = 0, scale = 0;
    cd P[129];
    for (int f = 0; f <= 128; ++f) {
      P[f] = 0;
      for (int j = 0; j < 256; ++j) P[f] += p[j] * std::polar(1.0, -2 * kPi * f * j / 256.0);
      scale = std::fmax(scale, std::abs(P[f]));
    }
    for (int l = 0; l < 8; ++l) {
      int k1a, k1b;
      mra::fwd_cols(l, k1a, k1b);
      float2 Za[8], Zb[8];
      for (int n2 = 0; n2 < 8; ++n2) { Za[n2] = Y[n2][k1a]; Zb[n2] = Y[n2][k1b]; }
      mra::dft8<-1>(Za);
      mra::dft8<-1>(Zb);
      int order[16], e = 0;
      mra::emit_slots(l, order);
      mra::fwd_emit(l, Za, Zb, tw256, [&](int slot, float a, float b) {
        check(e < 16 && order[e] == slot, "emit_slots order", e);
        ++e;
        if (slot == 0) {
          seen[0]++; seen[128]++;
          err = std::fmax(err, std::fabs(a - P[0].real()));
          err = std::fmax(err, std::fabs(b - P[128].real()));
        } else {
          seen[slot]++;
          err = std::fmax(err, std::abs(cd(a, b) - P[slot]));
        }
      });
    }
    for (int f = 0; f <= 128; ++f) check(seen[f] == 1, "fwd slot emitted once", seen[f]);
    check(err < 2e-6 * scale, "fwd ring fft", err / scale);
  }

  // ---- inverse over angle with the (a-b)(c-d) packing, both mirrors --------
  for (int rep = 0; rep < 10; ++rep) {
    const int R = 5;
    double p[R][256], q[R][256];
    for (int r = 0; r < R; ++r)
      for (int j = 0; j < 256; ++j) { p[r][j] = nd(rng); q[r][j] = nd(rng); }
    // direct sums: c0[a] = sum_r w_r sum_j p[j] q[j+a]; mirrored p1[j] = p[-j]
    double c0[256], c1[256], cmax = 0;
    for (int a = 0; a < 256; ++a) {
      c0[a] = c1[a] = 0;
      for (int r = 0; r < R; ++r)
        for (int j = 0; j < 256; ++j) {
          c0[a] += (r + 1) * p[r][j] * q[r][(j + a) & 255];
          c1[a] += (r + 1) * p[r][(256 - j) & 255] * q[r][(j + a) & 255];
        }
      cmax = std::fmax(cmax, std::fmax(std::fabs(c0[a]), std::fabs(c1[a])));
    }
    // spectra; reference side carries w_r / 256
    float2 V[256];
    double U[128][4] = {};
    for (int r = 0; r < R; ++r) {
      cd P[129], Q[129];
      for (int f = 0; f <= 128; ++f) {
        P[f] = Q[f] = 0;
        for (int j = 0; j < 256; ++j) {
          P[f] += p[r][j] * std::polar(1.0, -2 * kPi * f * j / 256.0);
          Q[f] += q[r][j] * std::polar(1.0, -2 * kPi * f * j / 256.0);
        }
        Q[f] *= (r + 1) / 256.0;
      }
      for (int s = 0; s < 128; ++s) {
        double a, b, c, d;
        if (s == 0) { a = P[0].real(); b = P[128].real(); c = Q[0].real(); d = Q[128].real(); }
        else { a = P[s].real(); b = P[s].imag(); c = Q[s].real(); d = Q[s].imag(); }
        U[s][0] += (a - b) * (c - d);  // U00
        U[s][1] += (a - b) * (c + d);  // U01
        U[s][2] += (a + b) * (c + d);  // U11
        U[s][3] += (a + b) * (c - d);  // U10
      }
    }
    // storage: logical j < 128 -> slot j (U00, U01); j >= 128 -> slot 256-j (U11, U10)
    for (int j = 0; j < 256; ++j) {
      int slot = j < 128 ? j : ((256 - j) & 127);
      V[j] = j < 128 ? make_float2((float)U[slot][0], (float)U[slot][1])
                     : make_float2((float)U[slot][2], (float)U[slot][3]);
    }
    for (int k2 = 0; k2 < 16; ++k2) {
      float2 x[16];
      for (int k1 = 0; k1 < 16; ++k1) x[k1] = V[16 * k1 + k2];
      mra::inv_pass1(k2, x, tw256);
      for (int n1 = 0; n1 < 16; ++n1) V[16 * n1 + k2] = x[n1];
    }
    double err = 0;
    for (int n1 = 0; n1 < 16; ++n1) {
      float2 x[16];
      for (int k2 = 0; k2 < 16; ++k2) x[k2] = V[16 * n1 + k2];
      mra::inv_pass2(x);
      for (int n2 = 0; n2 < 16; ++n2) {
        int a = n1 + 16 * n2;
        err = std::fmax(err, std::fabs(x[n2].x - c0[a]));
        err = std::fmax(err, std::fabs(x[n2].y - c1[a]));
      }
    }
    check(err < 2e-5 * cmax, "inverse over angle, both mirrors", err / cmax);
  }
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}
