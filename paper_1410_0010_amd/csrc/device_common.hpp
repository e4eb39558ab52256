// Device-side helpers: complex arithmetic, small DFTs and the LDS Stockham FFT
// used by every transform pass.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace apm {

template <typename T> struct vec;
template <> struct vec<float> { using c2 = float2; using c4 = float4; };
template <> struct vec<double> { using c2 = double2; using c4 = double4; };
template <typename T> using C2 = typename vec<T>::c2;
template <typename T> using V4 = typename vec<T>::c4;

// Tables reached through pointers stored in job records are in global memory, but
// the compiler cannot tell and would use flat loads, which count against the LDS
// wait counter too (an LDS wait then also waits for them).  Reading through a
// global-address-space pointer gives plain global loads.
template <typename T> using gptr = const __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> as_global(const void* p) {
  return (gptr<T>)p;
}
// writable counterpart, for stores and atomics through table pointers
template <typename T> using gmut = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gmut<T> as_global_mut(void* p) {
  return (gmut<T>)p;
}
// A descriptor struct copied out of global memory word by word through a global-space
// pointer: its fields become values (only the words used are loaded), read with
// global or scalar loads rather than generic ones.
template <typename S> __device__ __forceinline__ S load_global(const S* p) {
  static_assert(sizeof(S) % 4 == 0 && alignof(S) >= 4, "a struct of 4-byte words");
  S v;
  const gptr<uint32_t> src = as_global<uint32_t>(p);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) dst[i] = src[i];
  return v;
}
// relaxed device-scope atomic add through a global-address-space pointer
template <typename T> __device__ __forceinline__ T global_add(gmut<T> p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> using nvec2 = T __attribute__((ext_vector_type(2)));
template <typename T> using nvec4 = T __attribute__((ext_vector_type(4)));

template <typename T> __device__ __forceinline__ C2<T> mk(T x, T y) { C2<T> r; r.x = x; r.y = y; return r; }
// Marks a loaded value as used at this point (an empty asm statement: no instruction
// is emitted).  Placed after a batch of loads, it keeps the compiler from sinking
// each load into the loop iteration that consumes it, which would expose every
// load's latency on its own.
template <typename V> __device__ __forceinline__ void pin4(V& v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

// Cell c of a periodic axis of n cells, for c in [-1, n] (a periodic root's stencils).
__device__ __forceinline__ int wrap_cell(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// complex element i of a global table reached through a job record
template <typename T> __device__ __forceinline__ C2<T> load_c2(const void* base, int64_t i) {
  const nvec2<T> v = as_global<nvec2<T>>(base)[i];
  return mk<T>(v.x, v.y);
}
// element i of a global array of 4-vectors / int pairs reached through a table
template <typename T> __device__ __forceinline__ V4<T> load_v4(const void* base, int64_t i) {
  const nvec4<T> v = as_global<nvec4<T>>(base)[i];
  V4<T> r;
  r.x = v.x; r.y = v.y; r.z = v.z; r.w = v.w;
  return r;
}
__device__ __forceinline__ int2 load_i2(const void* base, int64_t i) {
  const nvec2<int> v = as_global<nvec2<int>>(base)[i];
  return make_int2(v.x, v.y);
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  C r; r.x = a.x * b.x + a.y * b.y; r.y = a.y * b.x - a.x * b.y; return r;
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot90(C a) {
  C r;
  if (INV) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}

template <int L> struct Log2 { static constexpr int v = 1 + Log2<L / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

// ---- small DFTs in registers (sign -1 forward, +1 inverse) ----------------------
template <bool INV, typename C> __device__ __forceinline__ void dft2(C* v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b); v[1] = csub(a, b);
}
template <bool INV, typename C> __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  C t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = rot90<INV>(csub(a1, a3));
  a0 = cadd(t0, t2); a2 = csub(t0, t2); a1 = cadd(t1, t3); a3 = csub(t1, t3);
}
template <bool INV, typename C> __device__ __forceinline__ void dft4(C* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }
template <bool INV, typename T> __device__ __forceinline__ void dft8(C2<T>* v) {
  // radix-2 split into even/odd 4-point DFTs, then combine with w8^k
  C2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  const T h = (T)0.70710678118654752440;   // 1/sqrt(2)
  // w8^1 = (1 -+ i)/sqrt2, w8^2 = -+i, w8^3 = (-1 -+ i)/sqrt2 (upper sign forward)
  C2<T> t1, t3;
  if (INV) {
    t1 = mk<T>(h * (o1.x - o1.y), h * (o1.x + o1.y));
    t3 = mk<T>(-h * (o3.x + o3.y), h * (o3.x - o3.y));
  } else {
    t1 = mk<T>(h * (o1.x + o1.y), h * (o1.y - o1.x));
    t3 = mk<T>(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  }
  C2<T> t2 = rot90<INV>(o2);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1); v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2); v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3); v[7] = csub(e3, t3);
}

// ---- XCD-aware block order -------------------------------------------------------
// The dispatcher hands workgroups to the 8 XCDs round-robin (block b to XCD b mod 8),
// and each XCD has its own L2.  Remapping so every XCD runs one contiguous range of
// logical blocks keeps neighbouring blocks -- which read the two halves of the same
// cache lines -- on one L2.  A bijection of [0, n) for any n.
constexpr int kXCD = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
  const int64_t q = n / kXCD, r = n % kXCD;
  const int64_t x = b % kXCD, i = b / kXCD;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---- synchronisation between Stockham stages -------------------------------------
// When a line's L/8 workers fit in one wavefront (L <= 512) its stages only exchange
// data inside that wavefront: an LDS fence plus a wavefront barrier orders them, and
// lines of other wavefronts are independent.  Longer lines need the block barrier.
template <int L> __device__ __forceinline__ void stage_sync() {
  if constexpr (L / 8 <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Cell (x, y, z) of flat index i (x fastest) in a box of nx by ny by any cells, with
// 32-bit arithmetic: every box of a plan has fewer than 2^31 cells (64-bit division is
// a long software sequence).
__device__ __forceinline__ void box_cell(int64_t i, int nx, int ny, int& x, int& y, int& z) {
  const uint32_t u = (uint32_t)i, row = u / (uint32_t)nx, zz = row / (uint32_t)ny;
  x = (int)(u - row * (uint32_t)nx);
  y = (int)(row - zz * (uint32_t)ny);
  z = (int)zz;
}

// ---- LDS layout of a row-pass line ------------------------------------------------
// In the transforms that run on lines held in LDS (fft_line, fft_line_rin: the x
// passes and the y transpose) element i of a line of length L sits at swz<L>(i) (an
// XOR permutation of the 8-value groups), and lines are line_stride(L) values apart.
// Both are chosen so the strided writes of the first Stockham stages and the
// contiguous reads spread over the LDS banks when a wavefront's lanes walk one line.
template <int L> __device__ __forceinline__ int swz(int i) {
  if constexpr (L >= 512) return i ^ (((i >> 3) & 7) ^ (((i >> 6) & 7) << 3));
  else if constexpr (L >= 32) return i ^ ((i >> 3) & (L / 8 - 1 < 63 ? L / 8 - 1 : 63));
  else return i;
}
__host__ __device__ constexpr int line_stride(int L) {
  return L == 16 ? 18 : L == 32 ? 37 : L == 64 ? 70 : L == 128 ? 133 : L == 256 ? 261
       : L == 512 ? 517 : L + 5;
}

// ---- LDS layout of a column-pass line ------------------------------------------------
// Transforms that start and end in registers (fft_regs) keep element i of a line at
// i + (i >> s): one spare slot after every 2^s elements, s = 3 (s = log2(L/8) for lines
// shorter than 64).  Every LDS access of their Stockham stages has the form base + o
// with o fixed for the stage, and for all of them pad(base + o) = pad(base) + o +
// (o >> s) (o is a multiple of 2^s, or base + o stays inside one aligned 2^s block): a
// worker forms one address per stage and its eight accesses take compile-time offsets.
// Lines are col_stride(L, nl) values apart, a stride the host picks so the nl lines a
// wavefront touches start on different banks.
template <int L> struct CPad {
  static constexpr int s = Log2<L / 8>::v < 3 ? Log2<L / 8>::v : 3;
  __device__ static __forceinline__ int at(int i) { return i + (i >> s); }
  static constexpr int off(int o) { return o + (o >> s); }
};
template <typename T> __host__ __device__ constexpr int col_stride(int L, int nl) {
  const int s = L >= 64 ? 3 : (L >= 32 ? 2 : 1);     // CPad<L>::s
  // 64 banks of 4 bytes: neighbouring lines start 64 / (dwords per value * nl) values
  // apart in bank order
  const int skew = 64 / ((int)(sizeof(T) / 2) * (nl > 0 ? nl : 1));
  return L + (L >> s) + (skew > 0 ? skew : 1);
}

// ---- twiddles ---------------------------------------------------------------------
// Every Stockham stage after the first is radix 8 with one butterfly per worker,
// k = w mod NS, and needs w_{8 NS}^{r k} for r = 1..7.  Only the base w_{8 NS}^k is
// read (once per kernel, beside the data loads, so no table read waits behind a
// barrier); the other powers are products of it, at most three deep.
template <typename T, int L> struct Twid {
  static constexpr int r0 = Log2<L>::v % 3;
  static constexpr int first_ns = r0 == 1 ? 2 : (r0 == 2 ? 4 : 8);   // NS of the first twiddled stage
  static constexpr int count() { int n = 0; for (int ns = first_ns; ns < L; ns *= 8) ++n; return n; }
  static constexpr int index(int ns) { int i = 0; for (int n = first_ns; n < ns; n *= 8) ++i; return i; }
  static constexpr int N = count();
  C2<T> t[N > 0 ? N : 1];
  __device__ __forceinline__ Twid(int w, const C2<T>* __restrict__ tw) {
    int ns = first_ns;
#pragma unroll
    for (int i = 0; i < N; ++i, ns *= 8) t[i] = tw[(w % ns) * (L / (ns * 8))];
  }
};

template <typename C>
__device__ __forceinline__ void twiddle_powers(C (&p)[8], C t1) {
  p[1] = t1;
  p[2] = cmul(p[1], p[1]);
  p[3] = cmul(p[2], p[1]);
  p[4] = cmul(p[2], p[2]);
  p[5] = cmul(p[4], p[1]);
  p[6] = cmul(p[3], p[3]);
  p[7] = cmul(p[4], p[3]);
}

// ---- Stockham auto-sort radix stages on one line held in LDS --------------------
// A line of L complex values; L/8 workers per line; each worker always handles
// 8 values per stage: one radix-8, two radix-4 or four radix-2 butterflies.
// Butterfly j of a stage with span NS reads line[j + r L/R], twiddles element r
// by w_{NS R}^{r (j mod NS)}, transforms, and writes line[(j/NS) NS R + j mod NS
// + r NS].  Twiddle bases in tb (Twid).
template <typename T, int L, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_stage(C2<T>* line, int w, const Twid<T, L>& tb) {
  constexpr int B = 8 / R;
  constexpr int W8 = L / 8;
  static_assert(NS == 1 || R == 8, "only a first stage has radix 2 or 4");
  C2<T> v[B][R];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int j = w + q * W8;
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = line[swz<L>(j + r * (L / R))];
    if constexpr (NS > 1) {
      C2<T> p[8];
      twiddle_powers(p, tb.t[Twid<T, L>::index(NS)]);
#pragma unroll
      for (int r = 1; r < 8; ++r) v[q][r] = INV ? cmulc(v[q][r], p[r]) : cmul(v[q][r], p[r]);
    }
    if (R == 8) dft8<INV, T>(v[q]);
    else if (R == 4) dft4<INV>(v[q]);
    else dft2<INV>(v[q]);
  }
  stage_sync<L>();
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int j = w + q * W8;
    const int k = j % NS;
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) line[swz<L>(base + r * NS)] = v[q][r];
  }
  stage_sync<L>();
}

template <typename T, int L, int NS, bool INV>
__device__ __forceinline__ void radix8_stages(C2<T>* line, int w, const Twid<T, L>& tb) {
  if constexpr (NS < L) {
    stockham_stage<T, L, 8, NS, INV>(line, w, tb);
    radix8_stages<T, L, NS * 8, INV>(line, w, tb);
  }
}

// Full in-place FFT of one LDS line (element i at line[swz<L>(i)]).  Every worker of the line must call it; for
// L > 512 it contains block barriers, so then every thread of the block must.
// The caller orders the line's LDS contents before (block barrier after a load
// with another thread mapping) and after it.  Unnormalised; INV: exp(+2 pi i ...).
template <typename T, int L, bool INV>
__device__ __forceinline__ void fft_line(C2<T>* line, int w, const Twid<T, L>& tb) {
  constexpr int p = Log2<L>::v;
  constexpr int r0 = p % 3;
  if constexpr (r0 == 1) {
    stockham_stage<T, L, 2, 1, INV>(line, w, tb);
    radix8_stages<T, L, 2, INV>(line, w, tb);
  } else if constexpr (r0 == 2) {
    stockham_stage<T, L, 4, 1, INV>(line, w, tb);
    radix8_stages<T, L, 4, INV>(line, w, tb);
  } else {
    radix8_stages<T, L, 1, INV>(line, w, tb);
  }
}

// ---- Stockham transform with the line in registers at both ends ------------------
// Worker w of a line holds elements w + m L/8 (m = 0..7) in v[] before and after the
// transform.  The first stage reads its butterflies' inputs from v (butterfly q of a
// stage of radix R takes elements w + (q + r B) L/8, B = 8/R) and the last stage
// writes its outputs back to the same places, so only the stages in between go
// through LDS.  The workers of a line may sit in different wavefronts (columns
// fastest across lanes, the layout of coalesced column loads), so the LDS exchanges
// use block barriers and every thread of the block must call this.  On entry no
// thread may still read the line's LDS; on exit reads of it may still be in flight:
// the caller puts a block barrier before the line's LDS is written again.  PAD picks
// the line layout: the padded one of CPad (lines col_stride apart) or the swizzled one
// of swz (lines line_stride apart); the z passes measured faster with the latter.

template <typename T, int L, int R, int NS, bool INV, bool FIRST, bool PAD>
__device__ __forceinline__ void regs_stage(C2<T>* line, int w, C2<T> (&v)[8], const Twid<T, L>& tb) {
  constexpr int B = 8 / R;
  constexpr int W8 = L / 8;
  constexpr bool LAST = NS * R == L;
  static_assert(NS == 1 || R == 8, "only a first stage has radix 2 or 4");
  C2<T> u[B][R];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int j = w + q * W8;
    if constexpr (FIRST) {
#pragma unroll
      for (int r = 0; r < R; ++r) u[q][r] = v[q + r * B];
    } else if constexpr (PAD) {
      const C2<T>* src = line + CPad<L>::at(j);
#pragma unroll
      for (int r = 0; r < R; ++r) u[q][r] = src[CPad<L>::off(r * (L / R))];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) u[q][r] = line[swz<L>(j + r * (L / R))];
    }
    if constexpr (NS > 1) {
      C2<T> p[8];
      twiddle_powers(p, tb.t[Twid<T, L>::index(NS)]);
#pragma unroll
      for (int r = 1; r < 8; ++r) u[q][r] = INV ? cmulc(u[q][r], p[r]) : cmul(u[q][r], p[r]);
    }
    if (R == 8) dft8<INV, T>(u[q]);
    else if (R == 4) dft4<INV>(u[q]);
    else dft2<INV>(u[q]);
  }
  if constexpr (LAST) {
    // j < NS here, so output r of butterfly q is element j + r NS = w + (q + r B) L/8
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * B] = u[q][r];
  } else {
    if constexpr (!FIRST) __syncthreads();           // this stage's reads are done
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int j = w + q * W8;
      const int base = (j / NS) * NS * R + j % NS;
      if constexpr (PAD) {
        C2<T>* dst = line + CPad<L>::at(base);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[CPad<L>::off(r * NS)] = u[q][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) line[swz<L>(base + r * NS)] = u[q][r];
      }
    }
    __syncthreads();                                 // writes seen by the next stage
  }
}

template <typename T, int L, int NS, bool INV, bool FIRST, bool PAD>
__device__ __forceinline__ void regs_radix8(C2<T>* line, int w, C2<T> (&v)[8], const Twid<T, L>& tb) {
  if constexpr (NS < L) {
    regs_stage<T, L, 8, NS, INV, FIRST, PAD>(line, w, v, tb);
    regs_radix8<T, L, NS * 8, INV, false, PAD>(line, w, v, tb);
  }
}

// Unnormalised; INV: exp(+2 pi i ...).  Same stage sequence as fft_line; tb from
// Twid<T, L>(w, tw) of the same worker.
template <typename T, int L, bool INV, bool PAD = true>
__device__ __forceinline__ void fft_regs(C2<T>* line, int w, C2<T> (&v)[8], const Twid<T, L>& tb) {
  constexpr int r0 = Log2<L>::v % 3;
  if constexpr (r0 == 1) {
    regs_stage<T, L, 2, 1, INV, true, PAD>(line, w, v, tb);
    regs_radix8<T, L, 2, INV, false, PAD>(line, w, v, tb);
  } else if constexpr (r0 == 2) {
    regs_stage<T, L, 4, 1, INV, true, PAD>(line, w, v, tb);
    regs_radix8<T, L, 4, INV, false, PAD>(line, w, v, tb);
  } else {
    regs_radix8<T, L, 1, INV, true, PAD>(line, w, v, tb);
  }
}

// fft_line with the line's elements w + m L/8 arriving in v[] (m = 0..7) instead of
// LDS: the first stage takes its inputs from the registers; the output is in LDS as
// for fft_line.  Same synchronisation as fft_line; the caller orders the LDS
// contents after it.
template <typename T, int L, bool INV>
__device__ __forceinline__ void fft_line_rin(C2<T>* line, int w, C2<T> (&v)[8], const Twid<T, L>& tb) {
  constexpr int r0 = Log2<L>::v % 3;
  constexpr int R = r0 == 1 ? 2 : (r0 == 2 ? 4 : 8);
  constexpr int B = 8 / R;
  constexpr int W8 = L / 8;
  static_assert(L > 8, "a single-stage line has no LDS stage");
#pragma unroll
  for (int q = 0; q < B; ++q) {
    C2<T> u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[q + r * B];
    if (R == 8) dft8<INV, T>(u);
    else if (R == 4) dft4<INV>(u);
    else dft2<INV>(u);
    const int j = w + q * W8;
#pragma unroll
    for (int r = 0; r < R; ++r) line[swz<L>(j * R + r)] = u[r];
  }
  stage_sync<L>();
  radix8_stages<T, L, R, INV>(line, w, tb);
}

// Lines per block for a given element type and length: 4096 (FP32) or 2048
// (FP64) complex values per block -> 32-33 KB of LDS, 256 or 512 threads.
template <typename T, int L> struct FFTShape {
  static constexpr int NL = (std::is_same<T, float>::value ? 4096 : 2048) / L;
  static constexpr int NT = NL * (L / 8);
  static constexpr int LS = L + 1;            // padded line stride in LDS
};

}  // namespace apm
