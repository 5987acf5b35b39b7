// Register-blocked Stockham FFT for power-of-two line lengths, used by the
// Hartley passes of the spectral Laplacian solve (see ccmf_dht.h for the
// method).  Everything that depends on the line length is a compile-time
// constant: each thread owns E elements of one complex line (thread t of a
// line holds positions t + TPL*e), performs E/R radix-R butterflies per stage
// in registers, and exchanges through LDS once per stage.
#pragma once

#include <hip/hip_runtime.h>

namespace ccmf {
namespace pow2 {

template <typename T>
struct CX {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ CX<T> add(CX<T> a, CX<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ CX<T> sub(CX<T> a, CX<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ CX<T> mul(CX<T> a, CX<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ CX<T> mi(CX<T> a) { return {a.y, -a.x}; }  // -i a
template <typename T>
__host__ __device__ __forceinline__ CX<T> pi(CX<T> a) { return {-a.y, a.x}; }  // +i a

// forward DFTs, X[p] = sum_r v[r] exp(-2 pi i p r / R)
template <typename T>
__host__ __device__ __forceinline__ void dft2(CX<T>* v) {
  const CX<T> a = v[0];
  v[0] = add(a, v[1]);
  v[1] = sub(a, v[1]);
}

template <typename T>
__host__ __device__ __forceinline__ void dft4(CX<T>* v) {
  const CX<T> a0 = add(v[0], v[2]), a1 = sub(v[0], v[2]);
  const CX<T> a2 = add(v[1], v[3]), a3 = sub(v[1], v[3]);
  v[0] = add(a0, a2);
  v[2] = sub(a0, a2);
  v[1] = add(a1, mi(a3));
  v[3] = add(a1, pi(a3));
}

template <typename T>
__host__ __device__ __forceinline__ void dft8(CX<T>* v) {
  CX<T> e[4] = {v[0], v[2], v[4], v[6]};
  CX<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
  const T h = T(0.70710678118654752440);
  o[1] = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};   // * W8^1
  o[2] = mi(o[2]);                                          // * W8^2
  o[3] = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};  // * W8^3
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    v[p] = add(e[p], o[p]);
    v[p + 4] = sub(e[p], o[p]);
  }
}

template <typename T>
__host__ __device__ __forceinline__ void dft16(CX<T>* v) {
  // 16 = 4 x 4: inner DFT4 over n1 for each n2, twiddle W16^(n2 k1), outer DFT4 over n2
  CX<T> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    CX<T> t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
    dft4(t);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
  }
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173), h = T(0.70710678118654752440);
  const CX<T> w1 = {c1, -s1}, w2 = {h, -h}, w3 = {s1, -c1}, w6 = {-h, -h}, w9 = {-c1, s1};
  y[1][1] = mul(y[1][1], w1);
  y[1][2] = mul(y[1][2], w2);
  y[1][3] = mul(y[1][3], w3);
  y[2][1] = mul(y[2][1], w2);
  y[2][2] = mi(y[2][2]);
  y[2][3] = mul(y[2][3], w6);
  y[3][1] = mul(y[3][1], w3);
  y[3][2] = mul(y[3][2], w6);
  y[3][3] = mul(y[3][3], w9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    CX<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4(t);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
  }
}

template <typename T, int R>
__host__ __device__ __forceinline__ void dft(CX<T>* v) {
  if constexpr (R == 2) dft2(v);
  if constexpr (R == 4) dft4(v);
  if constexpr (R == 8) dft8(v);
  if constexpr (R == 16) dft16(v);
}

// Stage plans: elements per thread E and radices R0..R3 (0 = no stage).
// Variant V = 0 uses the largest radices; V = 1 halves E where possible (more
// threads per line and fewer registers per thread); V = 2 uses E = 4 (radix-4
// stages, four times the threads of V = 0 for the same LDS tile) up to 256.
// Each pass uses a fixed variant (the launch code's variant_of).
template <int N, int V = 0>
struct Plan;
template <> struct Plan<2, 0>    { static constexpr int E = 2,  R0 = 2,  R1 = 0,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<4, 0>    { static constexpr int E = 4,  R0 = 4,  R1 = 0,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<8, 0>    { static constexpr int E = 8,  R0 = 8,  R1 = 0,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<16, 0>   { static constexpr int E = 16, R0 = 16, R1 = 0,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<32, 0>   { static constexpr int E = 8,  R0 = 8,  R1 = 4,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<64, 0>   { static constexpr int E = 8,  R0 = 8,  R1 = 8,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<128, 0>  { static constexpr int E = 16, R0 = 16, R1 = 8,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<256, 0>  { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<512, 0>  { static constexpr int E = 8,  R0 = 8,  R1 = 8,  R2 = 8; static constexpr int R3 = 0; };
template <> struct Plan<1024, 0> { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 4; static constexpr int R3 = 0; };
template <> struct Plan<2048, 0> { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 8; static constexpr int R3 = 0; };
template <> struct Plan<2, 1>    { static constexpr int E = 2,  R0 = 2,  R1 = 0,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<4, 1>    { static constexpr int E = 2,  R0 = 2,  R1 = 2,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<8, 1>    { static constexpr int E = 4,  R0 = 4,  R1 = 2,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<16, 1>   { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<32, 1>   { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 2; static constexpr int R3 = 0; };
template <> struct Plan<64, 1>   { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 4; static constexpr int R3 = 0; };
template <> struct Plan<128, 1>  { static constexpr int E = 8,  R0 = 8,  R1 = 8,  R2 = 2; static constexpr int R3 = 0; };
template <> struct Plan<256, 1>  { static constexpr int E = 8,  R0 = 8,  R1 = 8,  R2 = 4; static constexpr int R3 = 0; };
template <> struct Plan<512, 1>  { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 2; static constexpr int R3 = 0; };
template <> struct Plan<1024, 1> { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 4; static constexpr int R3 = 0; };
template <> struct Plan<2048, 1> { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 8; static constexpr int R3 = 0; };
template <> struct Plan<2, 2>    { static constexpr int E = 2,  R0 = 2,  R1 = 0,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<4, 2>    { static constexpr int E = 4,  R0 = 4,  R1 = 0,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<8, 2>    { static constexpr int E = 4,  R0 = 4,  R1 = 2,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<16, 2>   { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 0; static constexpr int R3 = 0; };
template <> struct Plan<32, 2>   { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 2; static constexpr int R3 = 0; };
template <> struct Plan<64, 2>   { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 4; static constexpr int R3 = 0; };
template <> struct Plan<128, 2>  { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 4; static constexpr int R3 = 2; };
template <> struct Plan<256, 2>  { static constexpr int E = 4,  R0 = 4,  R1 = 4,  R2 = 4; static constexpr int R3 = 4; };
template <> struct Plan<512, 2>  { static constexpr int E = 8,  R0 = 8,  R1 = 8,  R2 = 8; static constexpr int R3 = 0; };
template <> struct Plan<1024, 2> { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 4; static constexpr int R3 = 0; };
template <> struct Plan<2048, 2> { static constexpr int E = 16, R0 = 16, R1 = 16, R2 = 8; static constexpr int R3 = 0; };

// One Stockham stage on the E values a thread holds.  Before the stage thread t
// (0 <= t < TPL = N/E) holds x[t + TPL*e]; butterfly m of the thread (E/R of
// them) is u = t + TPL*m with inputs x[u + r*N/R] = element m + r*(E/R).
// Twiddles: W_N^(r * k * N/(Ns R)), k = u mod Ns, read from a stage-major table
// (stage_twiddle_index): the entries of one stage and one r are consecutive in
// k, so the lanes of a wavefront read consecutive LDS words (a plain table
// W_N^j read at stride r*k hits the same LDS bank from many lanes).
// Results go to position (u / Ns) * Ns * R + (u mod Ns) + r * Ns of the line.
// Position of W_N^(r k N/(NS R)) (1 <= r < R, 0 <= k < NS) in the stage-major
// table: the stages before this one hold sum (R_s - 1) NS_s = NS - 1 entries.
__host__ __device__ __forceinline__ constexpr int stage_twiddle_index(int NS, int r, int k) {
  return (NS - 1) + (r - 1) * NS + k;
}

template <typename T, int N, int E, int R, int NS>
__host__ __device__ __forceinline__ void stage_compute(CX<T>* v, int t, const CX<T>* __restrict__ tw) {
  constexpr int TPL = N / E;
  constexpr int BPT = E / R;
#pragma unroll
  for (int m = 0; m < BPT; ++m) {
    CX<T> b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) b[r] = v[m + r * BPT];
    if constexpr (NS > 1) {
      const int u = t + TPL * m;
      const int k = u & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) b[r] = mul(b[r], tw[stage_twiddle_index(NS, r, k)]);
    }
    dft<T, R>(b);
#pragma unroll
    for (int r = 0; r < R; ++r) v[m + r * BPT] = b[r];
  }
}

template <int N, int E, int R, int NS>
__host__ __device__ __forceinline__ int stage_out_pos(int t, int m, int r) {
  constexpr int TPL = N / E;
  const int u = t + TPL * m;
  return (u / NS) * NS * R + (u & (NS - 1)) + r * NS;
}

// Stage-major twiddle table of plan <N, V> from the plain table w[j] = W_N^j
// (interleaved re, im; n entries): out[2 idx], out[2 idx + 1] = W_N^(r k N/(NS R))
// at idx = stage_twiddle_index(NS, r, k).  N entries (the last one unused, zero).
template <int N, int V>
void stage_twiddles(const double* w, double* out) {
  using P = Plan<N, V>;
  const int radices[4] = {P::R0, P::R1, P::R2, P::R3};
  for (int j = 0; j < 2 * N; ++j) out[j] = 0.0;
  int ns = 1;
  for (int st = 0; st < 4 && radices[st] > 0; ++st) {
    const int R = radices[st];
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < ns; ++k) {
        const int idx = stage_twiddle_index(ns, r, k);
        const int j = r * k * (N / (ns * R));
        out[2 * idx] = w[2 * j];
        out[2 * idx + 1] = w[2 * j + 1];
      }
    ns *= R;
  }
}

}  // namespace pow2
}  // namespace ccmf
