// Device-side building blocks for LDS-staged Stockham FFTs on gfx950.
//
// A batch of P pencils of length N is processed by a workgroup; each pencil
// is owned by TPP = N / EPT threads and every thread keeps EPT complex
// elements in registers.  Between radix stages the data are exchanged through
// LDS; the first stage reads and the last stage writes the register layout
//     v[m] = x[t + TPP * m],   m = 0 .. EPT-1,
// so global loads and stores of consecutive t hit consecutive positions.
//
// The stage recurrence is the Stockham autosort form: at a stage of radix R
// after radices whose product is NS, butterfly j takes x[j + r N/R],
// multiplies by exp(-+2 pi i (j mod NS) r / (NS R)), applies the R-point DFT
// and writes to position (j / NS) NS R + (j mod NS) + r NS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pnp {

// builtin two-element vectors (assignable in every address space; loaded and
// stored as one 8- or 16-byte access)
typedef float cf32 __attribute__((ext_vector_type(2)));
typedef double cf64 __attribute__((ext_vector_type(2)));
template <typename T> struct cvec;
template <> struct cvec<float> { using type = cf32; };
template <> struct cvec<double> { using type = cf64; };
template <typename T> using cx = typename cvec<T>::type;

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by +i
template <typename T>
__device__ __forceinline__ cx<T> cmuli(cx<T> a) { return mk<T>(-a.y, a.x); }
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> cmulmi(cx<T> a) { return mk<T>(a.y, -a.x); }
// acc += a * s (real s)
template <typename T>
__device__ __forceinline__ void cfma(cx<T>& acc, cx<T> a, T s) {
  acc.x = fma(a.x, s, acc.x);
  acc.y = fma(a.y, s, acc.y);
}

// ---------------------------------------------------------------------------
// compile-time cos / sin of 2 pi a / b (Taylor series after exact octant
// reduction; accurate to about one unit in the last place of a double)
// ---------------------------------------------------------------------------
constexpr double kTwoPi = 6.283185307179586476925286766559;

constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) { term *= -x2 / ((2 * k - 1) * (2 * k)); sum += term; }
  return sum;
}
constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) { term *= -x2 / ((2 * k) * (2 * k + 1)); sum += term; }
  return sum;
}
// cos(2 pi r / b) for r / b in [0, 1/4]
constexpr double cos_quarter(long r, long b) {
  if (8 * r > b) return taylor_sin(kTwoPi * (double)(b - 4 * r) / (double)(4 * b));
  return taylor_cos(kTwoPi * (double)r / (double)b);
}
// cos(2 pi a / b) for integers, b > 0
constexpr double cos2pi(long a, long b) {
  long r = ((a % b) + b) % b;            // r / b in [0, 1)
  if (2 * r > b) r = b - r;              // even function: r / b in [0, 1/2]
  if (4 * r > b) return -cos_quarter(b - 2 * r, 2 * b);
  return cos_quarter(r, b);
}
constexpr double sin2pi(long a, long b) { return cos2pi(4 * a - b, 4 * b); }  // sin x = cos(x - pi/2)

// multiply by exp(s * 2 pi i * E / R) with s = -1 (forward) or +1 (inverse)
template <typename T, int E, int R, bool FWD>
__device__ __forceinline__ cx<T> twc(cx<T> a) {
  constexpr int e = ((E % R) + R) % R;
  constexpr int es = FWD ? (R - e) % R : e;    // exponent of exp(+2 pi i es / R)
  if constexpr (es == 0) {
    return a;
  } else if constexpr (4 * es == R) {
    return cmuli<T>(a);
  } else if constexpr (2 * es == R) {
    return mk<T>(-a.x, -a.y);
  } else if constexpr (4 * es == 3 * R) {
    return cmulmi<T>(a);
  } else {
    constexpr T c = (T)cos2pi(es, R);
    constexpr T s = (T)sin2pi(es, R);
    return mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// ---------------------------------------------------------------------------
// small DFTs in registers
// ---------------------------------------------------------------------------
template <typename T, int R, bool FWD> struct Dft;

template <typename T, bool FWD> struct Dft<T, 1, FWD> {
  static __device__ __forceinline__ void run(cx<T>*) {}
};

template <typename T, bool FWD> struct Dft<T, 2, FWD> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
  }
};

template <typename T, bool FWD> struct Dft<T, 3, FWD> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    constexpr T c = (T)-0.5;
    constexpr T s = (T)(FWD ? -0.86602540378443864676 : 0.86602540378443864676);
    cx<T> a = v[0], b = v[1], d = v[2];
    cx<T> t1 = cadd<T>(b, d);
    cx<T> t2 = mk<T>(a.x + c * t1.x, a.y + c * t1.y);
    cx<T> t3 = csub<T>(b, d);  // times i*s
    v[0] = cadd<T>(a, t1);
    v[1] = mk<T>(t2.x - s * t3.y, t2.y + s * t3.x);
    v[2] = mk<T>(t2.x + s * t3.y, t2.y - s * t3.x);
  }
};

template <typename T, bool FWD> struct Dft<T, 4, FWD> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a0 = cadd<T>(v[0], v[2]), a1 = csub<T>(v[0], v[2]);
    cx<T> b0 = cadd<T>(v[1], v[3]), b1 = csub<T>(v[1], v[3]);
    // forward: b1 * (-i); inverse: b1 * (+i)
    cx<T> b1r = FWD ? cmulmi<T>(b1) : cmuli<T>(b1);
    v[0] = cadd<T>(a0, b0);
    v[2] = csub<T>(a0, b0);
    v[1] = cadd<T>(a1, b1r);
    v[3] = csub<T>(a1, b1r);
  }
};

// R = R1 * R2 with input index m = R2 m1 + m2 and output index k = k1 + R1 k2
template <typename T, int R1, int R2, bool FWD> struct DftComposite {
  template <int M2>
  static __device__ __forceinline__ void col(const cx<T>* v, cx<T>* y) {
    cx<T> t[R1];
#pragma unroll
    for (int m1 = 0; m1 < R1; ++m1) t[m1] = v[R2 * m1 + M2];
    Dft<T, R1, FWD>::run(t);
    tw_row<M2, 0>(t, y);
  }
  template <int M2, int K1>
  static __device__ __forceinline__ void tw_row(const cx<T>* t, cx<T>* y) {
    if constexpr (K1 < R1) {
      y[M2 * R1 + K1] = twc<T, M2 * K1, R1 * R2, FWD>(t[K1]);
      tw_row<M2, K1 + 1>(t, y);
    }
  }
  template <int M2>
  static __device__ __forceinline__ void cols(const cx<T>* v, cx<T>* y) {
    if constexpr (M2 < R2) { col<M2>(v, y); cols<M2 + 1>(v, y); }
  }
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> y[R1 * R2];
    cols<0>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cx<T> t[R2];
#pragma unroll
      for (int m2 = 0; m2 < R2; ++m2) t[m2] = y[m2 * R1 + k1];
      Dft<T, R2, FWD>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
};

template <typename T, bool FWD> struct Dft<T, 6, FWD> : DftComposite<T, 2, 3, FWD> {};
template <typename T, bool FWD> struct Dft<T, 8, FWD> : DftComposite<T, 2, 4, FWD> {};
template <typename T, bool FWD> struct Dft<T, 12, FWD> : DftComposite<T, 3, 4, FWD> {};
template <typename T, bool FWD> struct Dft<T, 16, FWD> : DftComposite<T, 4, 4, FWD> {};

// ---------------------------------------------------------------------------
// radix plan: largest radix dividing both what is left of N and EPT
// ---------------------------------------------------------------------------
constexpr int pick_radix(int rem, int ept) {
  const int cand[7] = {16, 12, 8, 6, 4, 3, 2};
  for (int i = 0; i < 7; ++i)
    if (rem % cand[i] == 0 && ept % cand[i] == 0) return cand[i];
  return 1;
}

// Ordering of an LDS exchange.  WAVE = true when every lane that reads an
// element belongs to the wavefront that wrote it: LDS operations of one
// wavefront execute in issue order, so only compiler reordering has to be
// prevented (no s_barrier).  Otherwise the whole workgroup synchronises.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS view of one pencil: element pos lives at base[pos * es].  After the
// reads of an exchange the buffer must not be rewritten until every thread
// has read it: done() synchronises again.
template <typename T, bool WAVE = false> struct LdsPencil {
  cx<T>* base;
  int es;
  static constexpr bool wave = WAVE;
  __device__ __forceinline__ void st(int pos, cx<T> v) const { base[pos * es] = v; }
  __device__ __forceinline__ cx<T> ld(int pos) const { return base[pos * es]; }
  __device__ __forceinline__ void sync() const { lds_sync<WAVE>(); }
  __device__ __forceinline__ void done() const { lds_sync<WAVE>(); }
};

// The same view over two buffers used in turn: exchange e writes and reads
// buffer e mod 2, so the next exchange writes the other one and only one
// synchronisation per exchange is needed (a thread that writes buffer b again
// has passed the synchronisation of the exchange in between, which every
// thread reaches only after its reads of b).  Every thread of the workgroup
// must run the same sequence of exchanges.
template <typename T, bool WAVE = false> struct LdsPencil2 {
  cx<T>* base0;
  cx<T>* base1;
  int es;
  mutable int cur = 0;
  static constexpr bool wave = WAVE;
  __device__ __forceinline__ cx<T>* b() const { return cur ? base1 : base0; }
  __device__ __forceinline__ void st(int pos, cx<T> v) const { b()[pos * es] = v; }
  __device__ __forceinline__ cx<T> ld(int pos) const { return b()[pos * es]; }
  __device__ __forceinline__ void sync() const { lds_sync<WAVE>(); }
  __device__ __forceinline__ void done() const { cur ^= 1; }
};

// twiddle table tw[i] = exp(-2 pi i * i / N), i in [0, N), in LDS
template <typename T, int N, bool FWD>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* tw, int idx) {
  cx<T> w = tw[idx];
  return FWD ? w : cconj<T>(w);
}

// number of twiddles one thread applies in a full transform (stages after the first)
constexpr int tw_count(int n, int ept) {
  int c = 0;
  for (int ns = 1; ns < n;) {
    const int r = pick_radix(n / ns, ept);
    if (ns > 1) c += (ept / r) * (r - 1);
    ns *= r;
  }
  return c;
}
// index of the first twiddle of the stage that starts after radix product ns0
constexpr int tw_offset(int n, int ept, int ns0) {
  int c = 0;
  for (int ns = 1; ns < ns0;) {
    const int r = pick_radix(n / ns, ept);
    if (ns > 1) c += (ept / r) * (r - 1);
    ns *= r;
  }
  return c;
}

// The twiddles of one thread's share of a length-N transform, held in
// registers (filled once from the LDS table, reused for every field the
// thread transforms); forward values, conjugated for the inverse.
template <typename T, int N, int EPT>
struct TwReg {
  static constexpr int count = tw_count(N, EPT);
  cx<T> w[count > 0 ? count : 1];
  template <int NS, int OFF>
  __device__ __forceinline__ void fill(int t, const cx<T>* tab) {
    if constexpr (NS < N) {
      constexpr int R = pick_radix(N / NS, EPT);
      constexpr int B = EPT / R, TPP = N / EPT;
      if constexpr (NS > 1) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const int k = (t + TPP * b) % NS;
#pragma unroll
          for (int r = 1; r < R; ++r) w[OFF + b * (R - 1) + r - 1] = tab[k * r * (N / (NS * R))];
        }
        fill<NS * R, OFF + B * (R - 1)>(t, tab);
      } else {
        fill<NS * R, OFF>(t, tab);
      }
    }
  }
  __device__ __forceinline__ void load(int t, const cx<T>* tab) { fill<1, 0>(t, tab); }
};

template <typename T, int N, int EPT, int R, int NS, bool FWD>
__device__ __forceinline__ cx<T> stage_tw(const cx<T>* tw, int b, int r, int k) {
  return twiddle<T, N, FWD>(tw, k * r * (N / (NS * R)));
}
template <typename T, int N, int EPT, int R, int NS, bool FWD>
__device__ __forceinline__ cx<T> stage_tw(const TwReg<T, N, EPT>& tw, int b, int r, int) {
  const cx<T> w = tw.w[tw_offset(N, EPT, NS) + b * (R - 1) + r - 1];
  return FWD ? w : cconj<T>(w);
}

template <typename T, int N, int EPT, int R, int NS, bool FWD, class TW, class L>
__device__ __forceinline__ void stockham_stage(cx<T>* v, int t, const TW& tw, const L& lds) {
  constexpr int TPP = N / EPT;
  constexpr int B = EPT / R;
  static_assert(EPT % R == 0 && N % (NS * R) == 0, "bad radix plan");
  constexpr bool last = (NS * R == N);
  cx<T> out[EPT];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + TPP * b;
    cx<T> u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[b + r * B];
    if constexpr (NS > 1) {
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r)
        u[r] = cmul<T>(u[r], stage_tw<T, N, EPT, R, NS, FWD>(tw, b, r, k));
    }
    Dft<T, R, FWD>::run(u);
#pragma unroll
    for (int r = 0; r < R; ++r) out[b + r * B] = u[r];
  }
  if constexpr (last) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[m] = out[m];
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + TPP * b;
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) lds.st(base + r * NS, out[b + r * B]);
    }
    lds.sync();
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[m] = lds.ld(t + TPP * m);
    lds.done();
  }
}

template <typename T, int N, int EPT, int NS, bool FWD, class TW, class L>
__device__ __forceinline__ void stockham_run(cx<T>* v, int t, const TW& tw, const L& lds) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix(N / NS, EPT);
    static_assert(R > 1, "unsupported length / elements-per-thread pair");
    stockham_stage<T, N, EPT, R, NS, FWD>(v, t, tw, lds);
    stockham_run<T, N, EPT, NS * R, FWD>(v, t, tw, lds);
  }
}

// Unnormalised DFT of one pencil held as v[m] = x[t + (N/EPT) m].
// Every thread of the workgroup (or of the wavefront, for a wave-local LDS
// view) must call this: it contains the exchange synchronisation.
template <typename T, int N, int EPT, bool FWD, class TW, class L>
__device__ __forceinline__ void fft_pencil(cx<T>* v, int t, const TW& tw, const L& lds) {
  stockham_run<T, N, EPT, 1, FWD>(v, t, tw, lds);
}

}  // namespace pnp
