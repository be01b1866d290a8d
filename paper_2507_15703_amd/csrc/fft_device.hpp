// Complex arithmetic, radix-R inverse DFT butterflies and an LDS Stockham stage driver
// for gfx950 (wave64). Used by the three passes of the inverse 3-D FFT.
//
// Sign convention: every transform here is the unnormalised inverse DFT
//   y_k = sum_r v_r exp(+2 pi i r k / R),
// which composed over the stages gives T(j) = sum_f T(f) exp(+2 pi i f j / L).
#pragma once
#include <hip/hip_runtime.h>

namespace cmbx {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.y, a.x}; }  // i a
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------- butterflies
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T>
struct Dft<T, 3> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T h = T(0.8660254037844386467637231707529362);  // sqrt(3)/2
    cpx<T> s = v[1] + v[2], d = v[1] - v[2];
    cpx<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    cpx<T> j = {-h * d.y, h * d.x};  // i (sqrt3/2) d
    v[0] = v[0] + s;
    v[1] = m + j;
    v[2] = m - j;
  }
};

template <typename T>
__device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  cpx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_i(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <typename T>
struct Dft<T, 4> {
  static __device__ __forceinline__ void run(cpx<T>* v) { dft4(v[0], v[1], v[2], v[3]); }
};

template <typename T>
struct Dft<T, 8> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T c = T(0.7071067811865475244008443621048490);
    cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = {c * (o1.x - o1.y), c * (o1.x + o1.y)};    // x e^{i pi/4}
    o2 = mul_i(o2);                                  // x e^{i pi/2}
    o3 = {-c * (o3.x + o3.y), c * (o3.x - o3.y)};   // x e^{3 i pi/4}
    v[0] = e0 + o0; v[4] = e0 - o0;
    v[1] = e1 + o1; v[5] = e1 - o1;
    v[2] = e2 + o2; v[6] = e2 - o2;
    v[3] = e3 + o3; v[7] = e3 - o3;
  }
};

template <typename T>
struct Dft<T, 16> {
  // r = 4a + b, k = k1 + 4 k2: length-4 transforms over a, twiddles e^{2 pi i b k1 / 16},
  // then length-4 transforms over b.
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T c1 = T(0.9238795325112867561281831893967883);  // cos(pi/8)
    const T s1 = T(0.3826834323650897717284599840303989);  // sin(pi/8)
    const T c2 = T(0.7071067811865475244008443621048490);
    cpx<T> a[4][4];  // a[b][k1]
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      a[b][0] = v[b]; a[b][1] = v[4 + b]; a[b][2] = v[8 + b]; a[b][3] = v[12 + b];
      dft4(a[b][0], a[b][1], a[b][2], a[b][3]);
    }
    // b = 1: w^{k1}, k1 = 1,2,3 -> m = 1, 2, 3
    a[1][1] = cmul(a[1][1], cpx<T>{c1, s1});
    a[1][2] = cmul(a[1][2], cpx<T>{c2, c2});
    a[1][3] = cmul(a[1][3], cpx<T>{s1, c1});
    // b = 2: m = 2, 4, 6
    a[2][1] = cmul(a[2][1], cpx<T>{c2, c2});
    a[2][2] = mul_i(a[2][2]);
    a[2][3] = cmul(a[2][3], cpx<T>{-c2, c2});
    // b = 3: m = 3, 6, 9
    a[3][1] = cmul(a[3][1], cpx<T>{s1, c1});
    a[3][2] = cmul(a[3][2], cpx<T>{-c2, c2});
    a[3][3] = cmul(a[3][3], cpx<T>{-c1, -s1});
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<T> b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
      dft4(b0, b1, b2, b3);
      v[k1] = b0; v[k1 + 4] = b1; v[k1 + 8] = b2; v[k1 + 12] = b3;
    }
  }
};

// ---------------------------------------------------------------- stage plans
// Factorisation of a transform length L = 2^a 3^b into radix stages: radix-3 stages
// first, then the power of two. Plan P = 0 takes radix-8 stages with one radix-16, -4 or
// -2 stage to make up the remainder (a = 8 uses two radix-16 stages); plan P = 1 is an
// alternative ordering / split of the same power of two (e.g. 512 = 16 8 4 instead of
// 8 8 8, 256 = 4 8 8 instead of 16 16), chosen between them by the autotuner.
constexpr int kPlans = 2;
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
constexpr int pow3_count(int L) { return (L % 3 == 0) ? 1 + pow3_count(L / 3) : 0; }
constexpr int pow2_part(int L) { return (L % 3 == 0) ? pow2_part(L / 3) : L; }

constexpr int pow2_stage_count(int a, int P) {
  return a == 0 ? 0
       : a <= 4 ? 1
       : P == 1 ? (a <= 7 ? 2 : 3)
       : (a <= 8 ? 2 : 3);
}
constexpr int pow2_radix(int a, int i, int P) {
  // a: exponent of the power of two; i: stage index within the power-of-two stages
  return a <= 4 ? (1 << a)
       : P == 1 ? (a == 5 ? (i == 0 ? 4 : 8)
                 : a == 6 ? (i == 0 ? 4 : 16)
                 : a == 7 ? (i == 0 ? 8 : 16)
                 : a == 8 ? (i == 0 ? 4 : 8)
                 : a == 9 ? (i == 0 ? 16 : i == 1 ? 8 : 4)
                 : a == 10 ? (i == 0 ? 4 : 16)
                 : (i == 0 ? 8 : 16))  // a == 11
       : a == 5 ? (i == 0 ? 8 : 4)
       : a == 6 ? 8
       : a == 7 ? (i == 0 ? 16 : 8)
       : a == 8 ? 16
       : a == 9 ? 8
       : a == 10 ? (i == 0 ? 16 : 8)
       : (i < 2 ? 16 : 8);  // a == 11
}
constexpr int stage_count(int L, int P = 0) { return pow3_count(L) + pow2_stage_count(ilog2(pow2_part(L)), P); }
constexpr int stage_radix(int L, int i, int P = 0) {
  return i < pow3_count(L) ? 3 : pow2_radix(ilog2(pow2_part(L)), i - pow3_count(L), P);
}
constexpr int stage_stride(int L, int i, int P = 0) {
  return i == 0 ? 1 : stage_stride(L, i - 1, P) * stage_radix(L, i - 1, P);
}
constexpr int max_radix(int L, int P = 0, int i = 0) {
  return i == stage_count(L, P) ? 1
         : (stage_radix(L, i, P) > max_radix(L, P, i + 1) ? stage_radix(L, i, P) : max_radix(L, P, i + 1));
}
constexpr bool plan_ok(int L, int P = 0, int i = 0, int prod = 1) {
  return i == stage_count(L, P) ? prod == L : plan_ok(L, P, i + 1, prod * stage_radix(L, i, P));
}

// ---------------------------------------------------------------- stage driver
// One Stockham stage (radix R, stride NS = product of the earlier radices) over NSEQ
// independent sequences of length L. Each of the (L/R) NSEQ butterflies reads R inputs
// spaced L/R apart, multiplies input r by w^{r k} (k = j mod NS, w = e^{2 pi i/(NS R)}),
// transforms them and writes output r to position (j / NS) NS R + k + r NS. After the
// last stage the sequence is in natural order.
//
// Slot s -> (sequence, j): with SEQFAST consecutive lanes take consecutive sequences
// (column tiles, where the sequences are the contiguous dimension); otherwise consecutive
// j within one sequence (line tiles). src(seq, n) / dst(seq, n, v) access element n of a
// sequence. tw is the table of NTW-th roots exp(2 pi i m / NTW), NTW = L * TWMUL.
template <int L, int NSEQ, int NT, int R>
struct StageSlots {
  static constexpr int J = L / R;
  static constexpr int SLOTS = J * NSEQ;
  static constexpr int PER = (SLOTS + NT - 1) / NT;
  static constexpr bool FULL = (SLOTS % NT) == 0;
};

// The inputs of this thread's butterflies of a radix-R stage, v[q][r] = input r of slot
// tid + q NT (the slot mapping of fft_stage).
template <typename T, int L, int NSEQ, int NT, int R, bool SEQFAST, class Src>
__device__ __forceinline__ void stage_inputs(Src& src, cpx<T> (&v)[StageSlots<L, NSEQ, NT, R>::PER][R], int tid) {
  using SS = StageSlots<L, NSEQ, NT, R>;
#pragma unroll
  for (int q = 0; q < SS::PER; ++q) {
    const unsigned s = (unsigned)tid + q * NT;
    if (SS::FULL || s < (unsigned)SS::SLOTS) {
      const unsigned seq = SEQFAST ? s % NSEQ : s / SS::J;
      const unsigned j = SEQFAST ? s / NSEQ : s % SS::J;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src((int)seq, (int)(j + r * SS::J));
    }
  }
}

// Twiddles, butterflies and outputs of a radix-R stage (stride NS) on inputs in registers.
template <typename T, int L, int NSEQ, int NT, int R, int NS, bool SEQFAST, int TWMUL, class Dst>
__device__ __forceinline__ void stage_outputs(const cpx<T>* __restrict__ tw,
                                              cpx<T> (&v)[StageSlots<L, NSEQ, NT, R>::PER][R], Dst& dst, int tid) {
  using SS = StageSlots<L, NSEQ, NT, R>;
#pragma unroll
  for (int q = 0; q < SS::PER; ++q) {
    const unsigned s = (unsigned)tid + q * NT;
    if (SS::FULL || s < (unsigned)SS::SLOTS) {
      const unsigned seq = SEQFAST ? s % NSEQ : s / SS::J;
      const unsigned j = SEQFAST ? s / NSEQ : s % SS::J;
      const unsigned k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[r * k * (L / (NS * R)) * TWMUL]);
      }
      Dft<T, R>::run(v[q]);
      const unsigned base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst((int)seq, (int)(base + r * NS), v[q][r]);
    }
  }
  dst.done();
}

// (fft_stage keeps its own copy of the two halves: written through the helpers above, the
// noise + x pass took a few more VALU instructions for its addresses)
template <typename T, int L, int NSEQ, int NT, int R, int NS, bool SEQFAST, int TWMUL, class Src, class Dst>
__device__ __forceinline__ void fft_stage(const cpx<T>* __restrict__ tw, Src& src, Dst& dst, int tid) {
  constexpr int J = L / R;
  constexpr int SLOTS = J * NSEQ;
  constexpr int PER = (SLOTS + NT - 1) / NT;
  constexpr bool FULL = (SLOTS % NT) == 0;
  cpx<T> v[PER][R];
  // slot arithmetic unsigned: the thread index is not known to the compiler to be
  // non-negative, and signed division by the (power-of-two) constants costs fix-ups
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const unsigned s = (unsigned)tid + q * NT;
    if (FULL || s < (unsigned)SLOTS) {
      const unsigned seq = SEQFAST ? s % NSEQ : s / J;
      const unsigned j = SEQFAST ? s / NSEQ : s % J;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src((int)seq, (int)(j + r * J));
    }
  }
  src.done();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const unsigned s = (unsigned)tid + q * NT;
    if (FULL || s < (unsigned)SLOTS) {
      const unsigned seq = SEQFAST ? s % NSEQ : s / J;
      const unsigned j = SEQFAST ? s / NSEQ : s % J;
      const unsigned k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[r * k * (L / (NS * R)) * TWMUL]);
      }
      Dft<T, R>::run(v[q]);
      const unsigned base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst((int)seq, (int)(base + r * NS), v[q][r]);
    }
  }
  dst.done();
}

// LDS-resident sequences. SEQFAST layout: element n of sequence q in row sw(n), at
// sw(n) * NSEQ + q; otherwise at q * L + n. sw permutes the rows within aligned blocks of
// the first stage's radix R0 (a power of two): it flips the low bits of n by the bits
// above them, n ^ ((n / R0) & MASK). The first stage writes its output rows R0 apart, so
// without it the lanes of one write land on the same few of the 64 four-byte banks; with
// it the rows spread over the G = 256 B / row bytes row positions of a bank sweep. Reads,
// which run over consecutive rows, keep their banks. sw is the identity for a radix-3
// first stage.
// Workgroup barrier for LDS only: waits for the wave's own LDS accesses and then for the
// other waves, but not for its global memory operations, so that loads streaming into
// another LDS buffer (global_load_lds) stay in flight across it. (__syncthreads also
// waits for those.) The memory clobber keeps the compiler from moving memory accesses
// across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// LB: done() is lds_barrier instead of __syncthreads.
template <typename T, int L, int NSEQ, bool SEQFAST, int P = 0, bool LB = false>
struct LdsIO {
  static constexpr int R0 = stage_radix(L, 0, P);
  static constexpr bool POW2 = (R0 & (R0 - 1)) == 0;
  static constexpr int BANK_CPX = 256 / (int)sizeof(cpx<T>);  // complex values in one sweep of the banks
  // measured: the line layout (the z pass) runs slower permuted, so only rows are
  static constexpr int G = SEQFAST ? (NSEQ >= BANK_CPX ? 1 : BANK_CPX / NSEQ) : 1;
  static constexpr int MASK = POW2 ? (G < R0 ? G : R0) - 1 : 0;
  __device__ static __forceinline__ int sw(int n) { return MASK ? n ^ ((n / R0) & MASK) : n; }
  __device__ static __forceinline__ int index(int q, int n) { return SEQFAST ? sw(n) * NSEQ + q : q * L + sw(n); }
  cpx<T>* p;
  __device__ __forceinline__ cpx<T> operator()(int q, int n) const { return p[index(q, n)]; }
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const { p[index(q, n)] = v; }
  __device__ __forceinline__ void done() const {
    if constexpr (LB) lds_barrier();
    else __syncthreads();
  }
};

// LDS-resident lines (the line layout, not SEQFAST) with the elements of each aligned block
// of 32 permuted within it: element n of line q at q L + (n ^ ((n >> 3) & 3) ^
// (((n >> 5) & 7) << 2)) for lengths that are powers of two (a bijection on every aligned
// block of 32), q L + n otherwise. A stage writes its outputs R positions apart (4j + r,
// then 32 (j / 4) + j % 4 + 4 r, ...): in the natural layout 8 to 16 lanes of a wave then
// share a bank, here two (the least a 64-lane write of 8 bytes each takes); the reads,
// over consecutive j, stay at two. For 3 * 2^k the permutation helps none of the accesses
// and is not used.
template <typename T, int L, int NSEQ, bool LB = false>
struct LdsXorLines {
  static constexpr bool SW = (L & (L - 1)) == 0;
  static constexpr int perm(int n) { return SW ? n ^ ((n >> 3) & 3) ^ (((n >> 5) & 7) << 2) : n; }
  static constexpr bool bijective() {
    bool seen[L] = {};
    for (int n = 0; n < L; ++n) {
      const int m = perm(n);
      if (m < 0 || m >= L || seen[m]) return false;
      seen[m] = true;
    }
    return true;
  }
  static_assert(bijective(), "the line permutation must map [0, L) onto itself");
  __device__ static __forceinline__ int sw(int n) { return perm(n); }
  __device__ static __forceinline__ int index(int q, int n) { return q * L + sw(n); }
  cpx<T>* p;
  __device__ __forceinline__ cpx<T> operator()(int q, int n) const { return p[index(q, n)]; }
  __device__ __forceinline__ void operator()(int q, int n, cpx<T> v) const { p[index(q, n)] = v; }
  __device__ __forceinline__ void done() const {
    if constexpr (LB) lds_barrier();
    else __syncthreads();
  }
};

// Run all stages of a length-L transform with stage plan P: stage 0 reads from `first`,
// the last stage writes to `last`, stages in between go through the LDS sequences `lds`
// (laid out as Mid, by default LdsIO<T, L, NSEQ, SEQFAST, P>; LB: their barriers are
// lds_barrier). `tid` is the thread's index in the workgroup.
template <typename T, int L, int NSEQ, int NT, bool SEQFAST, int TWMUL, int S, class First, class Last, int P = 0,
          bool LB = false, class Mid = LdsIO<T, L, NSEQ, SEQFAST, P, LB>>
__device__ __forceinline__ void fft_run(const cpx<T>* __restrict__ tw, cpx<T>* lds, First& first, Last& last,
                                        int tid) {
  constexpr int NST = stage_count(L, P);
  static_assert(plan_ok(L, P), "unsupported transform length");
  if constexpr (S < NST) {
    constexpr int R = stage_radix(L, S, P);
    constexpr int NS = stage_stride(L, S, P);
    Mid mid{lds};
    if constexpr (S == 0 && NST == 1) {
      fft_stage<T, L, NSEQ, NT, R, NS, SEQFAST, TWMUL>(tw, first, last, tid);
    } else if constexpr (S == 0) {
      fft_stage<T, L, NSEQ, NT, R, NS, SEQFAST, TWMUL>(tw, first, mid, tid);
    } else if constexpr (S == NST - 1) {
      fft_stage<T, L, NSEQ, NT, R, NS, SEQFAST, TWMUL>(tw, mid, last, tid);
    } else {
      fft_stage<T, L, NSEQ, NT, R, NS, SEQFAST, TWMUL>(tw, mid, mid, tid);
    }
    fft_run<T, L, NSEQ, NT, SEQFAST, TWMUL, S + 1, First, Last, P, LB, Mid>(tw, lds, first, last, tid);
  }
}

// fft_run with the first stage's inputs already in registers (v, as stage_inputs loads
// them for stage plan P): callers that load the next transform's inputs while this one
// runs.
template <typename T, int L, int NSEQ, int NT, bool SEQFAST, int TWMUL, class Last, int P = 0, bool LB = false,
          class Mid = LdsIO<T, L, NSEQ, SEQFAST, P, LB>>
__device__ __forceinline__ void fft_run_from_regs(const cpx<T>* __restrict__ tw, cpx<T>* lds,
                                                  cpx<T> (&v)[StageSlots<L, NSEQ, NT, stage_radix(L, 0, P)>::PER]
                                                            [stage_radix(L, 0, P)],
                                                  Last& last, int tid) {
  constexpr int NST = stage_count(L, P);
  constexpr int R = stage_radix(L, 0, P);
  static_assert(plan_ok(L, P), "unsupported transform length");
  if constexpr (NST == 1) {
    stage_outputs<T, L, NSEQ, NT, R, 1, SEQFAST, TWMUL>(tw, v, last, tid);
  } else {
    Mid mid{lds};
    stage_outputs<T, L, NSEQ, NT, R, 1, SEQFAST, TWMUL>(tw, v, mid, tid);
    fft_run<T, L, NSEQ, NT, SEQFAST, TWMUL, 1, Mid, Last, P, LB, Mid>(tw, lds, mid, last, tid);
  }
}

}  // namespace cmbx
