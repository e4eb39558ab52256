// Transpose of the per-grid convolution (Sec. 2.2, Eq. 2, reversed): from the four
// field-box cotangents (a_x, a_y, a_z, Phi) of a grid to the cotangent of its GMF.
// The forward map is a real cyclic convolution on the zero-padded M box with
// Fourier multipliers -i d_i Gf (force) and Gp (potential); its transpose is the
// cyclic convolution with the flipped kernels, multipliers conj(-i d_i Gf) =
// +i d_i Gf and Gp, the four inputs summed into one output:
//
//   S(k) = Gf(k) [ i d_x X_x + i d_y X_y + i d_z X_z ](k) + Gp(k) X_Phi(k),
//   GMF_bar = GMF-box part of IDFT(S),  X_c = DFT(field-box cotangent c, zero padded).
//
// Because d_i depends only on k_i, each derivative is applied in the pass along its
// axis and the a_x / a_y / a_z terms are merged as early as possible.  The passes
// run the forward ones backwards, on the same buffers and job tables:
//   ax   field-box rows (4 components) -> half spectra; row pairs share a complex
//        FFT; +i d_x on component 0                         (y buffer: 4 arrays)
//   ay   columns along y: 4 lines -> FFT -> [X_x + i d_y X_y, X_z, X_Phi]  (z buffer)
//   az   columns along z: 3 FFTs -> S = Gf (U + i d_z V) + Gp P -> inverse FFT ->
//        the gz GMF planes                                   (spectrum buffer)
//   ayi  columns along y: inverse FFT, the gy GMF rows kept, in place
//   axi  GMF rows: Hermitian half spectra -> inverse real FFT, two rows per complex
//        FFT -> the gx GMF cells
// Unnormalised transforms; the kernel table carries 1/(Mx My Mz) as in the forward.
#include "apm_kernels.hpp"
#include "device_common.hpp"

namespace apm {

__device__ __forceinline__ int find_job_a(const ConvJob* __restrict__ jobs, int njobs, int64_t b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// (i d) z for real d
template <typename T> __device__ __forceinline__ C2<T> mul_id(T d, C2<T> z) {
  return mk<T>(-d * z.y, d * z.x);
}

// ------------------------------------------------------------------ ax ----------
// Block = nl/4 row pairs of the field box (rows r = j fy + y), 4 lines per pair (one
// per component): line = comp(row 2q) + i comp(row 2q + 1) at transform positions
// (ox + x) mod L.  Output: half spectra into the y buffer, rows of component c.
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_adj_x(const ConvJob* __restrict__ jobs, int njobs, int nl, AdjPtrs<T> ap,
        C2<T>* __restrict__ yb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int P = J.pitch;
  const int fx = J.f[0], fy = J.f[1], fz = J.f[2], ox = J.off[0];
  C2<T>* __restrict__ ybuf = yb + J.y_off;
  const gptr<T> dxs = as_global<T>(J.dsym[0]);
  const double* __restrict__ fb = ap.fbar[J.level] + 4 * J.fld_off;
  const int G = nl / 4;
  const int nt = nl * (L / 8);
  const int t = threadIdx.x;
  const Twid<T, L> tb(t % (L / 8), tw);   // line worker t mod L/8
  const int b = t / (L / 8), w = t % (L / 8);
  const int64_t rows = (int64_t)fz * fy;
  constexpr int LS = line_stride(L);
  for (int i = t; i < nl * LS; i += nt) lds[i] = mk<T>(0, 0);
  // each thread takes at most four cells (G 2 fx <= 4 nt since fx <= L); their 32 B
  // cotangent loads are all issued before the LDS stores
  V4<double> cv[4];
  int slot[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int idx = t + j * nt;
    slot[j] = -1;
    int64_t cell = 0;
    if (idx < G * 2 * fx) {
      const int gg = idx / (2 * fx), rem = idx % (2 * fx);
      const int half = rem / fx, x = rem % fx;
      const int64_t r = 2 * (blk * G + gg) + half;
      if (r < rows) {
        cell = r * fx + x;
        slot[j] = ((4 * gg) * LS + swz<L>((ox + x) & (L - 1))) * 2 + half;
      }
    }
    cv[j] = load_v4<double>(fb, cell);               // cell 0 when unused: a valid address
  }
  __syncthreads();                                   // the zeroing is done
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (slot[j] >= 0) {
      T* L0 = reinterpret_cast<T*>(lds) + slot[j];  // .x or .y of the line element
      L0[0] = (T)cv[j].x;
      L0[2 * LS] = (T)cv[j].y;
      L0[4 * LS] = (T)cv[j].z;
      L0[6 * LS] = (T)cv[j].w;
    }
  }
  __syncthreads();
  C2<T>* line = lds + b * LS;
  fft_line<T, L, false>(line, w, tb);
  const int64_t q = blk * G + b / 4;
  const int c = b & 3;
  const int64_t ra = 2 * q, rb = 2 * q + 1;
  if (ra < rows) {
    const int64_t cs = (int64_t)c * rows * P;
    C2<T>* outa = ybuf + cs + ra * P;
    C2<T>* outb = ybuf + cs + rb * P;
    const T h = (T)0.5;
    for (int k = w; k <= L / 2; k += L / 8) {
      const C2<T> z = line[swz<L>(k)], m = line[swz<L>((L - k) & (L - 1))];
      C2<T> A = mk<T>(h * (z.x + m.x), h * (z.y - m.y));
      C2<T> B = mk<T>(h * (z.y + m.y), h * (m.x - z.x));
      if (c == 0) {
        const T d = dxs[k];
        A = mul_id<T>(d, A);
        B = mul_id<T>(d, B);
      }
      outa[k] = A;
      if (rb < rows) outb[k] = B;
    }
  }
}

// ------------------------------------------------------------------ ay ----------
// Block = (plane j < fz, nl columns), 4 lines per column from the 4 y-buffer arrays
// (rows y < fy at positions (oy + y) mod L, zero elsewhere); forward FFT; writes
// U = X_x + i d_y X_y, V = X_z, P = X_Phi as z-buffer arrays 0, 1, 2 (all My rows).
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_adj_y(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls,
        const C2<T>* __restrict__ yb, C2<T>* __restrict__ zb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int W = J.M[0] / 2 + 1, My = J.M[1], P = J.pitch;
  const int fz = J.f[2], fy = J.f[1], oy = J.off[1];
  const int nbw = (W + nl - 1) / nl;
  const int j = (int)(blk / nbw);
  const int c0 = (int)(blk % nbw) * nl;
  const gptr<T> dys = as_global<T>(J.dsym[1]);
  const C2<T>* yin = yb + J.y_off + (int64_t)j * fy * P + c0;
  const int64_t ys = (int64_t)fz * fy * P;
  C2<T>* zout = zb + J.z_off + c0;                   // rows (j, k) at tile_row(j, k, fz)
  const int64_t zs = (int64_t)fz * My * P;
  const int t = threadIdx.x;
  const Twid<T, L> tb(t % (L / 8), tw);   // line worker t mod L/8
  const int cb = t % nl, r0 = t / nl;                // column-wise: rows r0 + q L/2
  const bool col_ok = c0 + cb < W;
  C2<T> v[2][4];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = r0 + q * (L / 2);                  // transform position
    const int y = (r - oy) & (L - 1);                // field row landing there
    const bool ok = col_ok && y < fy;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      v[q][a] = ok ? yin[a * ys + (int64_t)y * P + cb] : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = swz<L>(r0 + q * (L / 2));
#pragma unroll
    for (int a = 0; a < 4; ++a) lds[(a * nl + cb) * ls + r] = v[q][a];
  }
  __syncthreads();
  const int b = t / (L / 8), w = t % (L / 8);
  fft_line<T, L, false>(lds + b * ls, w, tb);
  __syncthreads();                                   // stores read four lines
  if (col_ok) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = r0 + q * (L / 2);
      const int ks = swz<L>(k);
      const T d = dys[k];
      const C2<T> X0 = lds[(0 * nl + cb) * ls + ks], X1 = lds[(1 * nl + cb) * ls + ks];
      const C2<T> U = cadd(X0, mul_id<T>(d, X1));
      const int64_t o = tile_row(j, k, fz) * P + cb;
      zout[o] = U;
      zout[zs + o] = lds[(2 * nl + cb) * ls + ks];
      zout[2 * zs + o] = lds[(3 * nl + cb) * ls + ks];
    }
  }
}

// ------------------------------------------------------------------ az ----------
// Block = (ky, nl columns), one line per column: the three z-buffer arrays in turn
// (planes j < fz at positions (oz + j) mod L) -> forward FFT -> accumulated into
// S = Gf (U + i d_z V) + Gp P in registers; then the inverse FFT of S and the gz GMF
// planes into the spectrum buffer.  Thread t is worker t / nl of column t mod nl,
// as in the forward z pass: loads and stores go straight to the transform registers.
template <typename T, int L>
__global__ void __launch_bounds__(kTwoSetThreads<T>)
k_adj_z(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls,
        const C2<T>* __restrict__ zb, C2<T>* __restrict__ specb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int W = J.M[0] / 2 + 1, My = J.M[1], P = J.pitch;
  const int gz = J.g[2], fz = J.f[2], oz = J.off[2];
  const int nbw = (W + nl - 1) / nl;
  const int ky = (int)(blk / nbw);
  const int c0 = (int)(blk % nbw) * nl;
  const C2<T>* zin = zb + J.z_off + tile_row(0, ky, fz) * P + c0;
  const int64_t pstride = (int64_t)kYT * P;            // next plane, same ky (tiled rows)
  const int64_t zs = (int64_t)fz * My * P;
  C2<T>* spec = specb + J.spec_off + tile_row(0, ky, gz) * P + c0;
  const gptr<T> dzs = as_global<T>(J.dsym[2]);
  const int t = threadIdx.x;
  const int cb = t % nl, w = t / nl;
  const Twid<T, L> tb(w, tw);
  const bool col_ok = c0 + cb < W;
  C2<T>* line = lds + cb * ls;
  const int kxc = col_ok ? c0 + cb : 0;
  const int kyo = ky <= My / 2 ? ky : My - ky;
  // 24-bit multiplies: jz < 2^11, kYT P < 2^24, every product < 2^31
  const uint32_t ps32 = (uint32_t)pstride;
  // multipliers of this column: its run of the tiled table (entries kOctKx apart);
  // each product's set is read where it is used (holding all three for the whole
  // kernel spills FP64 registers)
  // 32-bit offsets from a per-thread base (an octant table has < 2^31 values)
  const int64_t ks = J.kstride;                        // table values per entry
  const uint32_t kp = (uint32_t)J.kpot;                // Gp's offset in an entry
  const uint32_t ostride = (uint32_t)(kOctKx * ks);
  const gptr<T> gcol = as_global<T>(J.kern) + oct_col(kxc, kyo, J.M[0], L) * ks;
  // S accumulates in LDS, each thread's values in its own slots (no barrier: the same
  // thread reads them back), so the forward transforms do not hold it in registers
  C2<T>* ss = lds + (int64_t)nl * ls + t;
  const int nt = (int)blockDim.x;
#pragma unroll 1
  for (int s = 0; s < 3; ++s) {
    // the worker index, opaque to the compiler here: the addresses of the loads and
    // of the stages' LDS accesses are formed again in each pass of the loop instead of
    // held in registers across it
    int wr = w;
    asm volatile("" : "+v"(wr));
    const C2<T>* zs_in = zin + s * zs;
    C2<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = wr + q * (L / 8);                // transform position
      const int jz = (r - oz) & (L - 1);             // field plane landing there
      v[q] = (col_ok && jz < fz) ? zs_in[__umul24((uint32_t)jz, ps32) + cb] : mk<T>(0, 0);
    }
    if (s > 0) __syncthreads();                      // the previous transform's reads
    fft_regs<T, L, false, false>(line, wr, v, tb);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kz = wr + q * (L / 8);
      const int kzo = kz <= L / 2 ? kz : L - kz;
      const T gf = gcol[(uint32_t)kzo * ostride];
      const C2<T> X = v[q];
      if (s == 0) ss[q * nt] = mk<T>(gf * X.x, gf * X.y);
      else if (s == 1) ss[q * nt] = cadd(ss[q * nt], mul_id<T>(gf * dzs[kz], X));
      else {
        const T gp = gcol[(uint32_t)kzo * ostride + kp];
        ss[q * nt] = cadd(ss[q * nt], mk<T>(gp * X.x, gp * X.y));
      }
    }
  }
  C2<T> S[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) S[q] = ss[q * nt];
  __syncthreads();
  int wi = w;
  asm volatile("" : "+v"(wi));
  fft_regs<T, L, true, false>(line, wi, S, tb);
  if (col_ok) {
    C2<T>* dst = spec + w * pstride + cb;
    const int64_t qstride = (int64_t)(L / 8) * pstride;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int z = w + q * (L / 8);
      if (z < gz) dst[q * qstride] = S[q];
    }
  }
}

// ------------------------------------------------------------------ ayi ---------
// Block = (plane z < gz, nl columns): inverse FFT along y of all My rows, rows
// [0, gy) written back in place; thread t is worker t / nl of column t mod nl.
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_adj_y_inv(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls, C2<T>* __restrict__ specb,
            const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int W = J.M[0] / 2 + 1, gy = J.g[1], gz = J.g[2], P = J.pitch;
  const int nbw = (W + nl - 1) / nl;
  const int64_t p = blk / nbw;
  const int c0 = (int)(blk % nbw) * nl;
  C2<T>* base = specb + J.spec_off + c0;             // rows (p, r) at tile_row(p, r, gz)
  const int t = threadIdx.x;
  const int cb = t % nl, w = t / nl;
  const Twid<T, L> tb(w, tw);
  const bool col_ok = c0 + cb < W;
  C2<T> v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int r = w + q * (L / 8);
    v[q] = col_ok ? base[tile_row((int)p, r, gz) * P + cb] : mk<T>(0, 0);
  }
  fft_regs<T, L, true>(lds + cb * ls, w, v, tb);
  if (col_ok) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = w + q * (L / 8);
      if (r < gy) base[tile_row((int)p, r, gz) * P + cb] = v[q];
    }
  }
}

// ------------------------------------------------------------------ axi ---------
// Block = nl GMF row pairs (rows r = z gy + y): the two Hermitian half spectra form
// one complex line A + i B, whose inverse FFT has the two real rows as its real and
// imaginary parts; cells x < gx are written to the GMF cotangent.
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_adj_x_inv(const ConvJob* __restrict__ jobs, int njobs, int nl, AdjPtrs<T> ap,
            const C2<T>* __restrict__ specb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int gx = J.g[0], gy = J.g[1], gz = J.g[2], My = J.M[1], P = J.pitch;
  const C2<T>* __restrict__ spec = specb + J.spec_off;
  T* __restrict__ out = ap.gmf[J.level] + J.gmf_off;
  const int t = threadIdx.x;
  const Twid<T, L> tb(t % (L / 8), tw);   // line worker t mod L/8
  const int b = t / (L / 8), w = t % (L / 8);
  C2<T>* line = lds + b * line_stride(L);
  const int64_t rows = (int64_t)gy * gz;
  const int64_t q = blk * nl + b;
  const int64_t ra = 2 * q, rb = 2 * q + 1;
  if (ra < rows) {
    const bool hb = rb < rows;
    const int64_t za = ra / gy, ya = ra % gy, zb = hb ? rb / gy : za, yb = hb ? rb % gy : ya;
    const C2<T>* A = spec + tile_row((int)za, (int)ya, gz) * P;
    const C2<T>* B = spec + tile_row((int)zb, (int)yb, gz) * P;
    C2<T> av[8], bv[8];                              // all loads first
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = w + j * (L / 8);
      const int k = i <= L / 2 ? i : L - i;
      av[j] = A[k];
      bv[j] = B[k];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = w + j * (L / 8);
      const int k = i <= L / 2 ? i : L - i;
      C2<T> a = av[j], bq = hb ? bv[j] : mk<T>(0, 0);
      if (k == 0 || k == L / 2) { a.y = 0; bq.y = 0; }
      line[swz<L>(i)] = i <= L / 2 ? mk<T>(a.x - bq.y, a.y + bq.x) : mk<T>(a.x + bq.y, bq.x - a.y);
    }
  } else {
    for (int i = w; i < L; i += L / 8) line[swz<L>(i)] = mk<T>(0, 0);
  }
  __syncthreads();
  fft_line<T, L, true>(line, w, tb);
  if (ra < rows) {
    for (int x = w; x < gx; x += L / 8) {
      const C2<T> v = line[swz<L>(x)];
      out[ra * gx + x] = v.x;
      if (rb < rows) out[rb * gx + x] = v.y;
    }
  }
}

// ---------------------------------------------- potential-only transposes ------
// When the acceleration cotangents are all zero (a loss on potentials or on W only)
// the transposed convolution is the scalar one with Gp: one line per row / column.
//   apx  field-box rows of the Phi cotangent -> half spectra (y buffer array 0)
//   apy  columns along y (fy rows at (oy + y) mod L) -> FFT (z buffer array 0)
//   apz  columns along z (fz planes at (oz + j) mod L) -> FFT -> Gp -> inverse FFT
//        -> the gz GMF planes; then ayi and axi as above.
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_adjp_x(const ConvJob* __restrict__ jobs, int njobs, int nl, AdjPtrs<T> ap,
         C2<T>* __restrict__ yb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int P = J.pitch;
  const int fx = J.f[0], fy = J.f[1], fz = J.f[2], ox = J.off[0];
  C2<T>* __restrict__ ybuf = yb + J.y_off;
  const double* __restrict__ fb = ap.fbar[J.level] + J.fld_off;   // the Phi cotangent, dense
  const int t = threadIdx.x;
  const Twid<T, L> tb(t % (L / 8), tw);   // line worker t mod L/8
  const int b = t / (L / 8), w = t % (L / 8);
  C2<T>* line = lds + b * line_stride(L);
  const int64_t rows = (int64_t)fz * fy;
  const int64_t q = blk * nl + b;
  const int64_t ra = 2 * q, rb = 2 * q + 1;
  const bool hra = ra < rows, hrb = rb < rows;
  const double* fa = fb + (hra ? ra : 0) * fx;
  const double* fc = fb + (hrb ? rb : 0) * fx;
  double va[8], vb[8];                               // all loads first, clamped addresses
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int x = min((w + j * (L / 8) - ox) & (L - 1), fx - 1);
    va[j] = fa[x];
    vb[j] = fc[x];
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = w + j * (L / 8);
    const int x = (i - ox) & (L - 1);                // field cell landing at position i
    T xa = 0, xb = 0;
    if (x < fx) {
      if (hra) xa = (T)va[j];
      if (hrb) xb = (T)vb[j];
    }
    line[swz<L>(i)] = mk<T>(xa, xb);
  }
  __syncthreads();
  fft_line<T, L, false>(line, w, tb);
  if (ra < rows) {
    C2<T>* outa = ybuf + ra * P;
    C2<T>* outb = ybuf + rb * P;
    const T h = (T)0.5;
    for (int k = w; k <= L / 2; k += L / 8) {
      const C2<T> z = line[swz<L>(k)], m = line[swz<L>((L - k) & (L - 1))];
      outa[k] = mk<T>(h * (z.x + m.x), h * (z.y - m.y));
      if (rb < rows) outb[k] = mk<T>(h * (z.y + m.y), h * (m.x - z.x));
    }
  }
}

template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_adjp_y(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls,
         const C2<T>* __restrict__ yb, C2<T>* __restrict__ zb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int W = J.M[0] / 2 + 1, My = J.M[1], P = J.pitch;
  const int fy = J.f[1], fz = J.f[2], oy = J.off[1];
  const int nbw = (W + nl - 1) / nl;
  const int j = (int)(blk / nbw);
  const int c0 = (int)(blk % nbw) * nl;
  const C2<T>* yin = yb + J.y_off + (int64_t)j * fy * P + c0;
  C2<T>* zout = zb + J.z_off + c0;                   // rows (j, k) at tile_row(j, k, fz)
  const int t = threadIdx.x;
  const int cb = t % nl, w = t / nl;
  const Twid<T, L> tb(w, tw);
  const bool col_ok = c0 + cb < W;
  C2<T> v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int r = w + q * (L / 8);
    const int y = (r - oy) & (L - 1);
    v[q] = (col_ok && y < fy) ? yin[(int64_t)y * P + cb] : mk<T>(0, 0);
  }
  fft_regs<T, L, false>(lds + cb * ls, w, v, tb);
  if (col_ok) {
#pragma unroll
    for (int q = 0; q < 8; ++q) zout[tile_row(j, w + q * (L / 8), fz) * P + cb] = v[q];
  }
}

template <typename T, int L>
__global__ void __launch_bounds__(kTwoSetThreads<T>)
k_adjp_z(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls,
         const C2<T>* __restrict__ zb, C2<T>* __restrict__ specb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job_a(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int W = J.M[0] / 2 + 1, My = J.M[1], P = J.pitch;
  const int gz = J.g[2], fz = J.f[2], oz = J.off[2];
  const int nbw = (W + nl - 1) / nl;
  const int ky = (int)(blk / nbw);
  const int c0 = (int)(blk % nbw) * nl;
  const C2<T>* zin = zb + J.z_off + tile_row(0, ky, fz) * P + c0;
  const int64_t pstride = (int64_t)kYT * P;            // next plane, same ky (tiled rows)
  C2<T>* spec = specb + J.spec_off + tile_row(0, ky, gz) * P + c0;
  const int t = threadIdx.x;
  const int cb = t % nl, w = t / nl;
  const Twid<T, L> tb(w, tw);
  const bool col_ok = c0 + cb < W;
  C2<T>* line = lds + cb * ls;
  const int kxc = col_ok ? c0 + cb : 0;
  const int kyo = ky <= My / 2 ? ky : My - ky;
  // 24-bit multiplies: jz < 2^11, kYT P < 2^24, every product < 2^31
  const uint32_t ps32 = (uint32_t)pstride;
  const int64_t ks = J.kstride;                        // table values per entry
  const int64_t ostride = kOctKx * ks;                 // next |kz| of the column's run
  const gptr<T> gcol = as_global<T>(J.kern) + oct_col(kxc, kyo, J.M[0], L) * ks + J.kpot;
  C2<T> v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int r = w + q * (L / 8);
    const int jz = (r - oz) & (L - 1);
    v[q] = (col_ok && jz < fz) ? zin[__umul24((uint32_t)jz, ps32) + cb] : mk<T>(0, 0);
  }
  T gp[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kz = w + q * (L / 8);
    const int kzo = kz <= L / 2 ? kz : L - kz;
    gp[q] = gcol[kzo * ostride];
  }
  fft_regs<T, L, false, false>(line, w, v, tb);
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = mk<T>(gp[q] * v[q].x, gp[q] * v[q].y);
  __syncthreads();
  fft_regs<T, L, true, false>(line, w, v, tb);
  if (col_ok) {
    C2<T>* dst = spec + w * pstride + cb;
    const int64_t qstride = (int64_t)(L / 8) * pstride;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int z = w + q * (L / 8);
      if (z < gz) dst[q * qstride] = v[q];
    }
  }
}

#define APM_ADJ_DISPATCH(Lv, ...)                            \
  switch (Lv) {                                              \
    case 16: { constexpr int LL = 16; __VA_ARGS__; } break;   \
    case 32: { constexpr int LL = 32; __VA_ARGS__; } break;   \
    case 64: { constexpr int LL = 64; __VA_ARGS__; } break;   \
    case 128: { constexpr int LL = 128; __VA_ARGS__; } break; \
    case 256: { constexpr int LL = 256; __VA_ARGS__; } break; \
    case 512: { constexpr int LL = 512; __VA_ARGS__; } break; \
    case 1024: { constexpr int LL = 1024; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                    \
  }

template <typename T>
hipError_t launch_adj_pass(int pass, int L, int nl, const ConvJob* jobs, int njobs, int64_t nblocks,
                           const AdjPtrs<T>& ap, C2<T>* spec, C2<T>* zbuf, C2<T>* ybuf,
                           const void* tw, hipStream_t s) {
  if (njobs == 0 || nblocks == 0) return hipSuccess;
  const size_t shm = pass_lds<T>(pass, L, nl);
  if (shm == 0) return hipErrorInvalidConfiguration;
  const int ls = pass_row_stride<T>(pass, L, nl);
  const dim3 grid((unsigned)nblocks), block((unsigned)pass_threads(pass, L, nl));
  const C2<T>* twc = (const C2<T>*)tw;
  APM_ADJ_DISPATCH(L, {
    switch (pass) {
      case PASS_AX:
        hipLaunchKernelGGL((k_adj_x<T, LL>), grid, block, shm, s, jobs, njobs, nl, ap, ybuf, twc);
        break;
      case PASS_AY:
        hipLaunchKernelGGL((k_adj_y<T, LL>), grid, block, shm, s, jobs, njobs, nl, ls,
                           (const C2<T>*)ybuf, zbuf, twc);
        break;
      case PASS_AZ:
        hipLaunchKernelGGL((k_adj_z<T, LL>), grid, block, shm, s, jobs, njobs, nl, ls,
                           (const C2<T>*)zbuf, spec, twc);
        break;
      case PASS_AYI:
        hipLaunchKernelGGL((k_adj_y_inv<T, LL>), grid, block, shm, s, jobs, njobs, nl, ls, spec,
                           twc);
        break;
      case PASS_AXI:
        hipLaunchKernelGGL((k_adj_x_inv<T, LL>), grid, block, shm, s, jobs, njobs, nl, ap,
                           (const C2<T>*)spec, twc);
        break;
      case PASS_APX:
        hipLaunchKernelGGL((k_adjp_x<T, LL>), grid, block, shm, s, jobs, njobs, nl, ap, ybuf, twc);
        break;
      case PASS_APY:
        hipLaunchKernelGGL((k_adjp_y<T, LL>), grid, block, shm, s, jobs, njobs, nl, ls,
                           (const C2<T>*)ybuf, zbuf, twc);
        break;
      case PASS_APZ:
        hipLaunchKernelGGL((k_adjp_z<T, LL>), grid, block, shm, s, jobs, njobs, nl, ls,
                           (const C2<T>*)zbuf, spec, twc);
        break;
      default:
        return hipErrorInvalidValue;
    }
  });
  return hipGetLastError();
}

template <typename T, int L> static hipError_t allow_lds_adj() {
  const void* f[] = {(const void*)&k_adj_x<T, L>, (const void*)&k_adj_y<T, L>,
                     (const void*)&k_adj_z<T, L>, (const void*)&k_adj_y_inv<T, L>,
                     (const void*)&k_adj_x_inv<T, L>, (const void*)&k_adjp_x<T, L>,
                     (const void*)&k_adjp_y<T, L>, (const void*)&k_adjp_z<T, L>};
  for (const void* k : f) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLDS);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t allow_lds_adjoint() {
  hipError_t e = hipSuccess;
#define APM_ALLOW(LL)                                                         \
  if (e == hipSuccess) e = allow_lds_adj<float, LL>();                         \
  if (e == hipSuccess) e = allow_lds_adj<double, LL>();
  APM_ALLOW(16) APM_ALLOW(32) APM_ALLOW(64) APM_ALLOW(128) APM_ALLOW(256) APM_ALLOW(512)
  APM_ALLOW(1024)
#undef APM_ALLOW
  return e;
}

template hipError_t launch_adj_pass<float>(int, int, int, const ConvJob*, int, int64_t,
                                           const AdjPtrs<float>&, C2<float>*, C2<float>*,
                                           C2<float>*, const void*, hipStream_t);
template hipError_t launch_adj_pass<double>(int, int, int, const ConvJob*, int, int64_t,
                                            const AdjPtrs<double>&, C2<double>*, C2<double>*,
                                            C2<double>*, const void*, hipStream_t);

}  // namespace apm
