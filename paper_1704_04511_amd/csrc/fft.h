// Stockham autosort FFT building blocks for data staged in LDS (gfx950).
//
// A length-N transform is a sequence of radix-R passes (R in {2,3,4,5,8,16});
// pass s with radix R and current sub-transform length NS reads R elements at
// stride N/R, multiplies by the twiddles w^{r k}, k = j mod NS, w = e^{s 2 pi i / (NS R)},
// applies the R-point DFT in registers and writes them at stride NS starting at
// (j / NS) NS R + k.  After the last pass the output is in natural order.
// Passes run in place: every thread first pulls all of its butterflies into
// registers, the block synchronises, then the results are written back.
//
// LDS layout: element e of transform b sits at b * fft_stride(N) + fft_pidx(e),
// one unused slot after every 16 elements and one more per transform.  A first
// pass writes its outputs at stride R (16 elements = 128 bytes), which in an
// unpadded array puts a wave's stores on two of the 64 banks; padded, the
// strides become 17 and 34 banks apart.  The twiddles of each pass sit in a
// table [r][k] of their own, so the lanes of a butterfly row read consecutive
// entries.
#pragma once
#include "common.h"

// ------------------------------------------------ complex64 / complex128
// The passes below are written once for a complex type C (float2 or double2);
// the complex64 instances are the operator's transforms, the complex128 ones
// the adjoint half of the multichannel data term.
SLRX_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
SLRX_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
SLRX_DEV double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
SLRX_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
SLRX_DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
template <int SIGN> SLRX_DEV double2 cmul_i(double2 a) {
  return SIGN > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}
template <class C> struct Cx;
template <> struct Cx<float2> {
  using S = float;
  static SLRX_DEV float2 make(float x, float y) { return make_float2(x, y); }
  // sqrt(3)/2; cos, sin (2 pi/5), cos, sin (4 pi/5); cos/sin(pi j / 8), j = 0..7
  static constexpr float h3 = 0.86602540378443865f;
  static constexpr float c51 = 0.30901699437494742f, c52 = -0.80901699437494742f;
  static constexpr float s51 = 0.95105651629515357f, s52 = 0.58778525229247313f;
  static constexpr float r2 = 0.70710678118654752f;
  static SLRX_DEV float cs16(int j) {
    constexpr float t[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f,
                            0.0f, -0.38268343236508978f, -0.70710678118654752f, -0.92387953251128674f};
    return t[j];
  }
  static SLRX_DEV float sn16(int j) {
    constexpr float t[8] = {0.0f, 0.38268343236508978f, 0.70710678118654752f, 0.92387953251128674f,
                            1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f};
    return t[j];
  }
};
template <> struct Cx<double2> {
  using S = double;
  static SLRX_DEV double2 make(double x, double y) { return make_double2(x, y); }
  static constexpr double h3 = 0.86602540378443864676;
  static constexpr double c51 = 0.30901699437494742410, c52 = -0.80901699437494742410;
  static constexpr double s51 = 0.95105651629515357212, s52 = 0.58778525229247312917;
  static constexpr double r2 = 0.70710678118654752440;
  static SLRX_DEV double cs16(int j) {
    constexpr double t[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                             0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
    return t[j];
  }
  static SLRX_DEV double sn16(int j) {
    constexpr double t[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                             1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
    return t[j];
  }
};

// ------------------------------------------------------------ small DFTs
// X[k] = sum_j x[j] e^{SIGN 2 pi i j k / R}, in place on a register array.
template <int R, int SIGN> struct Dft;

template <int SIGN> struct Dft<2, SIGN> {
  template <class C> static SLRX_DEV void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN> struct Dft<4, SIGN> {
  template <class C> static SLRX_DEV void run(C* v) {
    C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    C a2 = cadd(v[1], v[3]), a3 = cmul_i<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
  }
};

template <int SIGN> struct Dft<3, SIGN> {
  template <class C> static SLRX_DEV void run(C* v) {
    using K = Cx<C>;
    using S = typename K::S;
    C t = cadd(v[1], v[2]);
    C d = cmul_i<SIGN>(cscale(csub(v[1], v[2]), K::h3));
    C m = csub(v[0], cscale(t, (S)0.5));
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, d);
    v[2] = csub(m, d);
  }
};

template <int SIGN> struct Dft<5, SIGN> {
  template <class C> static SLRX_DEV void run(C* v) {
    using K = Cx<C>;
    const auto c1 = K::c51, c2 = K::c52, s1 = K::s51, s2 = K::s52;
    C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    C x0 = v[0];
    C a1 = K::make(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
    C a2 = K::make(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
    C b1 = cmul_i<SIGN>(K::make(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
    C b2 = cmul_i<SIGN>(K::make(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// Radix 8 and 16 by one decimation-in-frequency split into two halves:
// X[2k] = DFT_{R/2}(x_j + x_{j+R/2}), X[2k+1] = DFT_{R/2}((x_j - x_{j+R/2}) w^j).
template <int SIGN> struct Dft<8, SIGN> {
  template <class C> static SLRX_DEV void run(C* v) {
    using K = Cx<C>;
    const auto c = K::r2;
    C a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = cadd(v[j], v[j + 4]);
      b[j] = csub(v[j], v[j + 4]);
    }
    // w8^j = e^{SIGN i pi j / 4}
    b[1] = cmul(b[1], K::make(c, SIGN * c));
    b[2] = cmul_i<SIGN>(b[2]);
    b[3] = cmul(b[3], K::make(-c, SIGN * c));
    Dft<4, SIGN>::run(a);
    Dft<4, SIGN>::run(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  }
};

template <int SIGN> struct Dft<16, SIGN> {
  template <class C> static SLRX_DEV void run(C* v) {
    using K = Cx<C>;
    C a[8], b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = cadd(v[j], v[j + 8]);
      C d = csub(v[j], v[j + 8]);
      b[j] = (j == 0) ? d : (j == 4) ? cmul_i<SIGN>(d) : cmul(d, K::make(K::cs16(j), SIGN * K::sn16(j)));
    }
    Dft<8, SIGN>::run(a);
    Dft<8, SIGN>::run(b);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  }
};

// ------------------------------------------------------------- FFT plans
template <int... Rs> struct Radices {};
template <int N> struct FftPlan;
template <> struct FftPlan<8> { using L = Radices<8>; };
template <> struct FftPlan<16> { using L = Radices<16>; };
template <> struct FftPlan<32> { using L = Radices<8, 4>; };
template <> struct FftPlan<64> { using L = Radices<16, 4>; };
template <> struct FftPlan<96> { using L = Radices<16, 3, 2>; };
template <> struct FftPlan<128> { using L = Radices<16, 8>; };
template <> struct FftPlan<160> { using L = Radices<16, 5, 2>; };
template <> struct FftPlan<192> { using L = Radices<16, 4, 3>; };
template <> struct FftPlan<256> { using L = Radices<16, 16>; };

SLRX_DEV int fft_pidx(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int fft_stride(int N) { return N + N / 16 + 1; }

// Twiddle table size: NS * R entries for every pass with NS > 1.
template <int NS, int... Rs> struct TwSize { static constexpr int v = 0; };
template <int NS, int R, int... Rest> struct TwSize<NS, R, Rest...> {
  static constexpr int v = (NS > 1 ? NS * R : 0) + TwSize<NS * R, Rest...>::v;
};
template <int N, int... Rs> constexpr int tw_size_of(Radices<Rs...>) { return TwSize<1, Rs...>::v; }
template <int N> constexpr int fft_tw_size() {
  constexpr int v = tw_size_of<N>(typename FftPlan<N>::L{});
  return v > 0 ? v : 1;
}

// Fill the per-pass tables from tw[t] = e^{-2 pi i t / N}: entry OFF + r NS + k
// of the pass (NS, R) is w^{r k} with w = e^{-2 pi i / (NS R)}.
template <int N, int NT, int OFF, int NS, int... Rs> struct TwFill {
  template <class C> static SLRX_DEV void run(C*, const C*) {}
};
template <int N, int NT, int OFF, int NS, int R, int... Rest> struct TwFill<N, NT, OFF, NS, R, Rest...> {
  template <class C> static SLRX_DEV void run(C* twt, const C* tw) {
    if (NS > 1)
      for (int i = threadIdx.x; i < NS * R; i += NT) {
        const int r = i / NS, k = i % NS;
        twt[OFF + i] = tw[r * k * (N / (NS * R))];
      }
    TwFill<N, NT, OFF + (NS > 1 ? NS * R : 0), NS * R, Rest...>::run(twt, tw);
  }
};
template <int N, int NT, class C, int... Rs> SLRX_DEV void tw_fill_of(C* twt, const C* tw, Radices<Rs...>) {
  TwFill<N, NT, 0, 1, Rs...>::run(twt, tw);
}
// Called by all NT threads; the tables are valid after the next barrier.
template <int N, int NT, class C> SLRX_DEV void fft_twiddles(C* twt, const C* tw) {
  tw_fill_of<N, NT>(twt, tw, typename FftPlan<N>::L{});
}

// One radix-R pass over nb <= MAXB transforms (transform index slowest across
// threads, butterfly index fastest).
template <int N, int R, int NS, int OFF, int SIGN, int MAXB, int NT, class C>
SLRX_DEV void fft_pass(C* lds, const C* twt, int nb) {
  constexpr int NBF = N / R;                 // butterflies per transform
  constexpr int MAXTOT = MAXB * NBF;
  constexpr int PER = (MAXTOT + NT - 1) / NT;
  constexpr int BS = fft_stride(N);
  const int tot = nb * NBF;
  C v[PER][R];
  int base[PER], jj[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * NT;
    const int bt = b / NBF, j = b % NBF;
    base[i] = bt * BS;
    jj[i] = j;
    if (b < tot) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[base[i] + fft_pidx(j + r * NBF)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * NT;
    if (b < tot) {
      const int j = jj[i];
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = twt[OFF + r * NS + k];
          if (SIGN > 0) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Dft<R, SIGN>::run(v[i]);
      const int o = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[base[i] + fft_pidx(o + r * NS)] = v[i][r];
    }
  }
  __syncthreads();
}

template <int N, int SIGN, int MAXB, int NT, int NS, int OFF, class C, int R, int... Rest>
SLRX_DEV void fft_passes(C* lds, const C* twt, int nb) {
  fft_pass<N, R, NS, OFF, SIGN, MAXB, NT>(lds, twt, nb);
  if constexpr (sizeof...(Rest) > 0)
    fft_passes<N, SIGN, MAXB, NT, NS * R, OFF + (NS > 1 ? NS * R : 0), C, Rest...>(lds, twt, nb);
}

template <int N, int SIGN, int MAXB, int NT, class C, int... Rs>
SLRX_DEV void fft_run(C* lds, const C* twt, int nb, Radices<Rs...>) {
  fft_passes<N, SIGN, MAXB, NT, 1, 0, C, Rs...>(lds, twt, nb);
}

// Unnormalised length-N DFTs (sign SIGN) of nb <= MAXB transforms held in LDS
// in the padded layout; twt holds the tables of fft_twiddles.  Must be called
// by all NT threads.
template <int N, int SIGN, int MAXB, int NT, class C>
SLRX_DEV void fft_lds(C* lds, const C* twt, int nb) {
  fft_run<N, SIGN, MAXB, NT>(lds, twt, nb, typename FftPlan<N>::L{});
}

// Rows r0 .. r0+RB-1 of the frame at offset fo, each the sum of `groups`
// planes of the transposed layout (plane g at g * gstride, entry (row r,
// column c) at c P + r), added in plane order, into LDS rows, then their
// forward row DFTs of length N.  Called by all NT threads; twt must have been
// filled before the call (the first barrier here orders it).
template <int N, int MAXB, int NT, class C>
SLRX_DEV void rows_sum_fwd(C* lds, const C* twt, const C* d, int groups, long gstride, long fo, int P, int r0,
                           int RB) {
  constexpr int BS = fft_stride(N);
  for (int e = threadIdx.x; e < RB * N; e += NT) {  // consecutive threads walk a column
    const long src = fo + (long)(e / RB) * P + r0 + e % RB;
    C v = d[src];
    for (int g = 1; g < groups; ++g) v = cadd(v, d[(long)g * gstride + src]);
    lds[(e % RB) * BS + fft_pidx(e / RB)] = v;
  }
  __syncthreads();
  fft_lds<N, -1, MAXB, NT>(lds, twt, RB);
}

// Host dispatch of a launch template over the supported transform lengths.
#define SLRX_DISPATCH_N(n, F, ...)            \
  switch (n) {                                \
    case 8: return F<8>(__VA_ARGS__);         \
    case 16: return F<16>(__VA_ARGS__);       \
    case 32: return F<32>(__VA_ARGS__);       \
    case 64: return F<64>(__VA_ARGS__);       \
    case 96: return F<96>(__VA_ARGS__);       \
    case 128: return F<128>(__VA_ARGS__);     \
    case 160: return F<160>(__VA_ARGS__);     \
    case 192: return F<192>(__VA_ARGS__);     \
    case 256: return F<256>(__VA_ARGS__);     \
  }                                           \
  return hipErrorInvalidValue;
