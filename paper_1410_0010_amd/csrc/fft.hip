// Transform passes of the per-grid convolution (Sec. 2.2, Eq. 2): a real 3-D FFT of
// the zero-padded GMF, multiplication by the influence functions with Fourier-space
// differencing, and the inverse transforms of the four outputs (a_x, a_y, a_z, Phi).
//
// Spectrum layout (complex, x fastest): planes z, rows y (My of them), columns
// kx in [0, W), W = Mx/2 + 1, rows P = pitch apart (W rounded up to 16 values, so
// a block's column segment never straddles more cache lines than it must).  Five passes per grid:
//   x_fwd   GMF rows (gx reals, zero-padded to Mx) -> half spectra, two real rows
//           per complex FFT                                   (gy*gz rows)
//   y_fwd   columns along y: gy inputs -> My outputs, in place (gz planes)
//   z_conv  columns along z: gz inputs -> Mz-point forward FFT -> times three
//           multipliers (Gf, -i d_z Gf, Gp) -> three inverse FFTs -> fz outputs each
//   y_inv   columns along y: the three z outputs -> four lines per column (a_x from
//           Gf, a_y = -i d_y Gf, a_z, Phi) -> My-point inverse FFTs -> fy outputs
//           (the x and y derivatives are applied where d_x, d_y vary along the
//           line: in the x and y inverse passes; along z they are constants)
//   x_inv   two rows of one component per complex inverse FFT, Hermitian rows ->
//           real field-box rows, written as 4-vectors per cell (fy*fz rows)
// With one kernel for force and potential (spectral gradient: Gp = Gf) the potential
// is the a_x line before its x derivative: the z pass writes two arrays (Gf rho,
// -i d_z Gf rho), the y inverse pass three lines per column (a_x / Phi, a_y, a_z),
// and the x inverse pass takes both a_x (with -i d_x) and Phi from the first.
// Zero planes/rows of the padding are never read or transformed twice: y_fwd reads
// only gy rows, z_conv only gz planes, and the inverse passes write only the field
// box.  Unnormalised transforms; 1/(Mx My Mz) is folded into the kernel table.
//
// Batching: each pass is one launch per line length L over any set of grids (all
// grids of all levels in apm_solve: the levels' convolutions are independent).  A
// job table lists the grids with the index of their first block; a block finds its
// grid by binary search.  Lines per block (nl) is a launch parameter, chosen by the
// autotuner per (pass, L, precision).
#include <type_traits>

#include "apm_kernels.hpp"
#include "device_common.hpp"

namespace apm {

// Block -> job: last job whose first block is <= b (jobs sorted by blk0).
__device__ __forceinline__ int find_job(const ConvJob* __restrict__ jobs, int njobs, int64_t b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ x forward --
// Job = one grid; block = nl row pairs of its GMF (rows r = z gy + y).
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_fft_x_fwd(const ConvJob* __restrict__ jobs, int njobs, int nl, LevelPtrs<T> lp,
            C2<T>* __restrict__ specb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int gx = J.g[0], gy = J.g[1], gz = J.g[2], My = J.M[1], P = J.pitch;
  const T* __restrict__ gmf = lp.gmf[J.level] + J.gmf_off;
  C2<T>* __restrict__ spec = specb + J.spec_off;
  const int t = threadIdx.x;
  const Twid<T, L> tb(t % (L / 8), tw);   // line worker t mod L/8
  const int b = t / (L / 8), w = t % (L / 8);
  C2<T>* line = lds + b * line_stride(L);
  const int64_t rows = (int64_t)gy * gz;
  const int64_t q = blk * nl + b;
  const int64_t ra = 2 * q, rb = 2 * q + 1;
  // a subgrid of a periodic plan convolves its GMF minus the average density (on the
  // GMF box only; the padding stays zero), the difference formed in FP64
  const bool sub = J.mean != nullptr;
  const double mu = sub ? as_global<double>(J.mean)[0] : 0.0;
  // loads first, from clamped (valid) addresses, then the zero padding is selected
  const bool hra = ra < rows, hrb = rb < rows;
  const T* rowa = gmf + (hra ? ra : 0) * gx;
  const T* rowb = gmf + (hrb ? rb : 0) * gx;
  T va[8], vb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = min(w + j * (L / 8), gx - 1);
    va[j] = rowa[i];
    vb[j] = rowb[i];
  }
  C2<T> v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = w + j * (L / 8);
    T xa = 0, xb = 0;
    if (i < gx) {
      if (hra) xa = sub ? (T)((double)va[j] - mu) : va[j];
      if (hrb) xb = sub ? (T)((double)vb[j] - mu) : vb[j];
    }
    v[j] = mk<T>(xa, xb);
  }
  fft_line_rin<T, L, false>(line, w, v, tb);
  if (ra < rows) {
    const int64_t za = ra / gy, ya = ra % gy, zb = rb / gy, yb = rb % gy;
    C2<T>* outa = spec + tile_row((int)za, (int)ya, gz) * P;
    C2<T>* outb = spec + tile_row((int)zb, (int)yb, gz) * P;
    const T h = (T)0.5;
    for (int k = w; k <= L / 2; k += L / 8) {
      C2<T> z = line[swz<L>(k)], m = line[swz<L>((L - k) & (L - 1))];
      outa[k] = mk<T>(h * (z.x + m.x), h * (z.y - m.y));
      if (rb < rows) outb[k] = mk<T>(h * (z.y + m.y), h * (m.x - z.x));
    }
  }
}

// ------------------------------------------------------ y forward (columns) --
// Lines along y of the gz spectrum planes: rows [0, gy) in, all My rows out, in place.
// Thread t is worker t / nl of column t mod nl: the coalesced column loads and
// stores go straight to and from the transform's registers.
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_fft_y_fwd(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls, C2<T>* __restrict__ specb,
            const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job(jobs, njobs, gb)];
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
    v[q] = (r < gy && col_ok) ? base[tile_row((int)p, r, gz) * P + cb] : mk<T>(0, 0);
  }
  fft_regs<T, L, false>(lds + cb * ls, w, v, tb);
  if (col_ok) {
#pragma unroll
    for (int q = 0; q < 8; ++q) base[tile_row((int)p, w + q * (L / 8), gz) * P + cb] = v[q];
  }
}

// --------------------------------------------------------- z pass + multiply --
// For one (ky, block of kx) of a grid: forward FFT along z of the gz non-zero
// planes, then three products and inverse FFTs, written as arrays s = 0, 1, 2 of
// the z buffer (planes s fz + j, rows ky, columns kx):
//   s = 0: Gf(k) rho_hat            (the x and y derivatives follow in later passes)
//   s = 1: -i d_z(k_z) Gf(k) rho_hat
//   s = 2: Gp(k) rho_hat
// kern: octant table of (Gf, Gp), index ((|kz| Oy) + |ky|) W + kx, already scaled.
// Thread t works on column t mod nl as worker t / nl of its line: the column loads
// and stores are coalesced across lanes and go straight to and from the registers
// the transforms start and end in (only the middle Stockham stages use LDS).

// KS: kernel-table values per octant entry (2: (Gf, Gp) pairs, 1: Gf alone, whose
// potential product is then array 0 itself and is not written).
template <typename T, int L, int KS>
__global__ void __launch_bounds__(kTwoSetThreads<T>)
k_fft_z_conv(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls,
             const C2<T>* __restrict__ specb, C2<T>* __restrict__ zb,
             const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int W = J.M[0] / 2 + 1, My = J.M[1], P = J.pitch;
  const int gz = J.g[2], fz = J.f[2], oz = J.off[2];
  const int nbw = (W + nl - 1) / nl;
  const int ky = (int)(blk / nbw);
  const int c0 = (int)(blk % nbw) * nl;
  const C2<T>* __restrict__ spec = specb + J.spec_off;
  C2<T>* __restrict__ zo = zb + J.z_off;
  const gptr<T> dzs = as_global<T>(J.dsym[2]);
  const int64_t pstride = (int64_t)kYT * P;            // next plane, same ky (tiled rows)
  const int64_t qstride = (int64_t)(L / 8) * pstride;   // uniform: q steps by a scalar
  const int t = threadIdx.x;
  const int cb = t % nl, w = t / nl;
  const Twid<T, L> tb(w, tw);
  const bool col_ok = c0 + cb < W;
  C2<T>* line = lds + cb * ls;
  C2<T> X[8];
  {
    const C2<T>* src = spec + tile_row(0, ky, gz) * P + c0 + cb + w * pstride;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int z = w + q * (L / 8);
      X[q] = (z < gz && col_ok) ? src[q * qstride] : mk<T>(0, 0);
    }
  }
  // multipliers of this column: its run of the tiled table, kz after kz, beside the
  // runs of the block's neighbouring columns
  const int kxc = col_ok ? c0 + cb : 0;
  const int kyo = ky <= My / 2 ? ky : My - ky;
  using TV = typename std::conditional<KS == 2, nvec2<T>, T>::type;
  const gptr<TV> gcol = as_global<TV>(J.kern) + oct_col(kxc, kyo, J.M[0], L);
  // with one kernel the multiplier is read once, while the forward transform runs,
  // and the slots below hold Gf X: both products are formed from them
  T gf[KS == 1 ? 8 : 1];
  if constexpr (KS == 1) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kz = w + q * (L / 8);
      const int kzo = kz <= L / 2 ? kz : L - kz;
      gf[q] = gcol[(uint32_t)kzo * kOctKx];
    }
  }
  fft_regs<T, L, false, false>(line, w, X, tb);
  // the forward result waits in LDS, each thread's own values in its own slots (no
  // barrier: the same thread reads them back), so the inverse transforms do not
  // hold it in registers
  C2<T>* xs = lds + (int64_t)nl * ls + t;
  const int nt = (int)blockDim.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if constexpr (KS == 1) xs[q * nt] = mk<T>(gf[q] * X[q].x, gf[q] * X[q].y);
    else xs[q * nt] = X[q];
  }
  const int64_t zas = (int64_t)fz * My * P;            // stride between z arrays
  C2<T>* dst = zo + tile_row(0, ky, fz) * P + c0 + cb;
  constexpr int kProducts = KS == 1 ? 2 : 3;        // arrays written
#pragma unroll 1
  for (int s = 0; s < kProducts; ++s) {
    C2<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kz = w + q * (L / 8);
      const C2<T> x = xs[q * nt];
      T mul;
      if constexpr (KS == 2) {
        const int kzo = kz <= L / 2 ? kz : L - kz;
        const TV gv = gcol[(uint32_t)kzo * kOctKx];
        mul = s == 0 ? gv.x : (s == 1 ? dzs[kz] * gv.x : gv.y);
      } else {
        mul = s == 0 ? (T)1 : dzs[kz];
      }
      v[q] = s == 1 ? mk<T>(mul * x.y, -mul * x.x)   // -i d_z Gf X
                    : mk<T>(mul * x.x, mul * x.y);
    }
    __syncthreads();                                 // the previous transform's reads
    // the worker index, opaque to the compiler here: the LDS addresses of the stages
    // are formed again in each product instead of held in registers across the loop
    int wr = w;
    asm volatile("" : "+v"(wr));
    fft_regs<T, L, true, false>(line, wr, v, tb);
    if (col_ok) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = (w + q * (L / 8) - oz) & (L - 1);  // field plane of element w + q L/8
        if (j < fz) dst[s * zas + j * pstride] = v[q];
      }
    }
  }
}

// -------------------------------------------------------- y inverse (columns) --
// Block = (plane j < fz, nl columns): NC lines per column built from one read of
// the z arrays: a_x <- Gf rho (its x derivative follows in the x pass),
// a_y <- -i d_y(k_y) Gf rho, a_z <- array 1, and with NC = 4 Phi <- array 2 (with
// NC = 3 the potential is the a_x line itself); inverse FFT along y; rows j' < fy
// written from transform index (off_y + j') mod L into the y buffer (planes c fz + j,
// fy rows, W columns).  Thread t is worker t / nl of column t mod nl and transforms
// the column's lines one after another: its column loads and stores go straight to
// and from the transform's registers, a block covers nl adjacent columns of every
// row it touches, and array 0 is read once for the a_x and a_y lines.
template <typename T, int L, int NC>
__global__ void __launch_bounds__(kTwoSetThreads<T>)
k_fft_y_inv(const ConvJob* __restrict__ jobs, int njobs, int nl, int ls,
            const C2<T>* __restrict__ zb, C2<T>* __restrict__ yb, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int W = J.M[0] / 2 + 1, My = J.M[1], P = J.pitch;
  const int fz = J.f[2], fy = J.f[1], oy = J.off[1];
  const int nbw = (W + nl - 1) / nl;
  const int j = (int)(blk / nbw);
  const int c0 = (int)(blk % nbw) * nl;
  const gptr<T> dys = as_global<T>(J.dsym[1]);
  const int t = threadIdx.x;
  const int cb = t % nl, w = t / nl;
  const Twid<T, L> tb(w, tw);
  const bool col_ok = c0 + cb < W;
  const int64_t zs = (int64_t)fz * My * P;             // stride between z arrays
  const C2<T>* zin = zb + J.z_off + c0 + cb;
  C2<T>* line = lds + cb * ls;
  // arrays 0 and 1, both read before the first transform
  C2<T> a0[8], a1[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t o = tile_row(j, w + q * (L / 8), fz) * P;
    a0[q] = col_ok ? zin[o] : mk<T>(0, 0);
    a1[q] = col_ok ? zin[zs + o] : mk<T>(0, 0);
  }
  const int64_t ys = (int64_t)fz * fy * P;             // stride between components
  C2<T>* yout = yb + J.y_off + (int64_t)j * fy * P + c0 + cb;
#pragma unroll 1
  for (int c = 0; c < NC; ++c) {
    // the worker index, opaque to the compiler here: the addresses of the stages' LDS
    // accesses and of the stores are formed again for each line instead of held in
    // registers across the loop
    int wr = w;
    asm volatile("" : "+v"(wr));
    C2<T> v[8];
    if (c == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = a0[q];
    } else if (c == 1) {                             // -i d_y Gf rho
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const T d = dys[wr + q * (L / 8)];
        v[q] = mk<T>(d * a0[q].y, -d * a0[q].x);
      }
    } else if (c == 2) {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = a1[q];
    } else {                                         // NC = 4: Phi from array 2
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = col_ok ? zin[2 * zs + tile_row(j, wr + q * (L / 8), fz) * P] : mk<T>(0, 0);
    }
    if (c > 0) __syncthreads();                      // the previous line's LDS reads
    fft_regs<T, L, true>(line, wr, v, tb);
    if (col_ok) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int jj = (wr + q * (L / 8) - oy) & (L - 1);  // field row of this element
        if (jj < fy) yout[c * ys + (int64_t)jj * P] = v[q];
      }
    }
  }
}

// ------------------------------------------------------------------ x inverse --
// Flattened output rows r = j fy + y (j < fz, y < fy) are taken in pairs (2q, 2q+1);
// each component c of a pair is one complex line A_c(row 2q) + i A_c(row 2q+1) with
// Hermitian completion, so the real and imaginary parts of the inverse FFT are the
// two rows.  Pairing rows of the same component keeps magnitudes alike (an
// acceleration and the potential can differ by 1/dx, and a shared complex FFT would
// hand the larger one's rounding to the smaller).  Component 0 gets its x
// derivative here: A_0(k) -> -i d_x(k) A_0(k).  4 lines per row pair; writes
// field[r fx + x] = (a_x, a_y, a_z, Phi).  Rows are contiguous: no LDS padding.
template <typename T, int L>
__global__ void __launch_bounds__(1024)
k_fft_x_inv(const ConvJob* __restrict__ jobs, int njobs, int nl, const C2<T>* __restrict__ yb,
            LevelPtrs<T> lp, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
  const ConvJob& J = jobs[find_job(jobs, njobs, gb)];
  const int64_t blk = gb - J.blk0;
  const int P = J.pitch;
  const int fx = J.f[0], fy = J.f[1], fz = J.f[2], ox = J.off[0];
  const C2<T>* __restrict__ ybuf = yb + J.y_off;
  const gptr<T> dxs = as_global<T>(J.dsym[0]);
  V4<T>* __restrict__ field = lp.fld[J.level] + J.fld_off;
  const int G = nl / 4;
  const int nt = nl * (L / 8);
  const int t = threadIdx.x;
  const Twid<T, L> tb(t % (L / 8), tw);   // line worker t mod L/8
  const int b = t / (L / 8), w = t % (L / 8);
  const int64_t rows = (int64_t)fz * fy;
  const int64_t q = blk * G + b / 4;
  const int c = b & 3;
  const int64_t ra = 2 * q, rb = 2 * q + 1;
  constexpr int LS = line_stride(L);
  C2<T>* line = lds + b * LS;
  C2<T> v[8];
  if (ra < rows) {
    // with one kernel for force and potential, Phi is the a_x rows without d_x
    const int src = (c == 3 && J.kstride == 1) ? 0 : c;
    const int64_t cs = (int64_t)src * rows * P;       // component stride
    const C2<T>* A = ybuf + cs + ra * P;
    const bool hb = rb < rows;
    const C2<T>* B = ybuf + cs + (hb ? rb : ra) * P;
    // all eight elements' loads are issued before any is used (a loop that stores to
    // LDS after each load waits out one HBM round trip per element)
    C2<T> av[8], bv[8];
    T dv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = w + j * (L / 8);
      const int k = i <= L / 2 ? i : L - i;
      av[j] = A[k];
      bv[j] = B[k];
      dv[j] = dxs[k];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = w + j * (L / 8);
      const int k = i <= L / 2 ? i : L - i;
      C2<T> a = av[j], bq = hb ? bv[j] : mk<T>(0, 0);
      if (c == 0) {
        const T d = dv[j];
        a = mk<T>(d * a.y, -d * a.x);
        bq = mk<T>(d * bq.y, -d * bq.x);
      }
      if (k == 0 || k == L / 2) { a.y = 0; bq.y = 0; }
      v[j] = i <= L / 2 ? mk<T>(a.x - bq.y, a.y + bq.x) : mk<T>(a.x + bq.y, bq.x - a.y);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = mk<T>(0, 0);
  }
  fft_line_rin<T, L, true>(line, w, v, tb);
  __syncthreads();                                   // stores read four lines
  for (int idx = t; idx < G * 2 * fx; idx += nt) {
    const int gg = idx / (2 * fx), rem = idx % (2 * fx);
    const int half = rem / fx, x = rem % fx;
    const int64_t r = 2 * (blk * G + gg) + half;
    if (r < rows) {
      const int xi = swz<L>((ox + x) & (L - 1));
      const C2<T>* L0 = lds + (4 * gg) * LS + xi;
      V4<T> o;
      if (half == 0) {
        o.x = L0[0].x; o.y = L0[LS].x; o.z = L0[2 * LS].x; o.w = L0[3 * LS].x;
      } else {
        o.x = L0[0].y; o.y = L0[LS].y; o.z = L0[2 * LS].y; o.w = L0[3 * LS].y;
      }
      field[r * fx + x] = o;
    }
  }
}

// ------------------------------------------------------------------ launchers --
int64_t pass_blocks(int pass, const int g[3], const int M[3], const int f[3], int nl) {
  const int64_t W = M[0] / 2 + 1;
  const int64_t nbw = (W + nl - 1) / nl;
  // potential-only transposes: the forward x / y pass shapes over the field box
  if (pass == PASS_APX) return (((int64_t)f[1] * f[2] + 1) / 2 + nl - 1) / nl;
  if (pass == PASS_APY) return nbw * f[2];
  pass = mirror_pass(pass);
  switch (pass) {
    case PASS_X_FWD: return (((int64_t)g[1] * g[2] + 1) / 2 + nl - 1) / nl;
    case PASS_Y_FWD: return nbw * g[2];
    case PASS_Z_CONV: return nbw * M[1];
    case PASS_Y_INV: return nbw * f[2];
    case PASS_X_INV: return (((int64_t)f[1] * f[2] + 1) / 2 + nl / 4 - 1) / (nl / 4);
  }
  return 0;
}

template <typename T> int default_lines(int pass, int L) {
  const bool mirror = mirror_pass(pass) != pass;
  pass = mirror_pass(pass);
  int nl = (std::is_same<T, float>::value ? 4096 : 2048) / L;
  if (pass == PASS_X_INV) return nl < 4 ? 4 : nl;
  if (pass == PASS_Y_INV && mirror) return nl / 4 < 1 ? 1 : nl / 4;
  if (pass == PASS_Z_CONV) while (nl > 1 && nl * (L / 8) > kTwoSetThreads<T>) nl /= 2;
  return nl;
}

static int pass_lines_per_block(int pass, int nl, int nc) {
  // the y inverse pass transforms its nc lines per column one after another; its
  // transpose holds all four at once
  (void)nc;
  if (pass == PASS_Y_INV) return nl;
  return mirror_pass(pass) == PASS_Y_INV ? 4 * nl : nl;
}

// LDS line stride: line_stride(L) for the passes on swizzled lines (the row passes'
// fft_line and the z passes), col_stride(L, nl) for the y passes (the padded layout
// of fft_regs; also room enough for the swizzled lines of the y transpose).
template <typename T> static int pass_ls(int pass, int L, int nl) {
  const int m = mirror_pass(pass);
  return m == PASS_Y_FWD || m == PASS_Y_INV ? col_stride<T>(L, nl) : line_stride(L);
}

template <typename T> int pass_row_stride(int pass, int L, int nl) { return pass_ls<T>(pass, L, nl); }
int pass_threads(int pass, int L, int nl, int nc) {
  return pass_lines_per_block(pass, nl, nc) * (L / 8);
}

template <typename T> size_t pass_lds(int pass, int L, int nl, int nc) {
  if (nl < 1 || (nc != 3 && nc != 4)) return 0;
  const int lines = pass_lines_per_block(pass, nl, nc);
  // the z passes and the forward y inverse pass hold two sets of line values per thread
  const bool two_sets = pass == PASS_Y_INV || mirror_pass(pass) == PASS_Z_CONV;
  pass = mirror_pass(pass);
  // the z pass also parks each thread's eight forward-transform values (nl L values)
  const size_t bytes = ((size_t)lines * pass_ls<T>(pass, L, nl) + (pass == PASS_Z_CONV ? (size_t)nl * L : 0)) *
                       sizeof(C2<T>);
  const int max_threads = two_sets ? kTwoSetThreads<T> : 1024;
  if (lines * (L / 8) > max_threads || bytes > (size_t)kMaxLDS) return 0;
  if (pass == PASS_X_INV && (nl % 4) != 0) return 0;
  return bytes;
}

#define APM_FFT_DISPATCH(Lv, ...)                            \
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
hipError_t launch_pass(int pass, int L, int nl, int nc, const ConvJob* jobs, int njobs,
                       int64_t nblocks, const LevelPtrs<T>& lp, C2<T>* spec, C2<T>* zbuf,
                       C2<T>* ybuf, const void* tw, hipStream_t s) {
  if (njobs == 0 || nblocks == 0) return hipSuccess;
  const size_t shm = pass_lds<T>(pass, L, nl, nc);
  if (shm == 0) return hipErrorInvalidConfiguration;
  const int ls = pass_ls<T>(pass, L, nl);
  const dim3 grid((unsigned)nblocks), block((unsigned)(pass_lines_per_block(pass, nl, nc) * (L / 8)));
  const C2<T>* twc = (const C2<T>*)tw;
  APM_FFT_DISPATCH(L, {
    switch (pass) {
      case PASS_X_FWD:
        hipLaunchKernelGGL((k_fft_x_fwd<T, LL>), grid, block, shm, s, jobs, njobs, nl, lp, spec, twc);
        break;
      case PASS_Y_FWD:
        hipLaunchKernelGGL((k_fft_y_fwd<T, LL>), grid, block, shm, s, jobs, njobs, nl, ls, spec, twc);
        break;
      case PASS_Z_CONV:                    // nc == 3: single-kernel tables
        if (nc == 3)
          hipLaunchKernelGGL((k_fft_z_conv<T, LL, 1>), grid, block, shm, s, jobs, njobs, nl, ls,
                             (const C2<T>*)spec, zbuf, twc);
        else
          hipLaunchKernelGGL((k_fft_z_conv<T, LL, 2>), grid, block, shm, s, jobs, njobs, nl, ls,
                             (const C2<T>*)spec, zbuf, twc);
        break;
      case PASS_Y_INV:
        if (nc == 3)
          hipLaunchKernelGGL((k_fft_y_inv<T, LL, 3>), grid, block, shm, s, jobs, njobs, nl, ls,
                             (const C2<T>*)zbuf, ybuf, twc);
        else
          hipLaunchKernelGGL((k_fft_y_inv<T, LL, 4>), grid, block, shm, s, jobs, njobs, nl, ls,
                             (const C2<T>*)zbuf, ybuf, twc);
        break;
      case PASS_X_INV:
        hipLaunchKernelGGL((k_fft_x_inv<T, LL>), grid, block, shm, s, jobs, njobs, nl,
                           (const C2<T>*)ybuf, lp, twc);
        break;
      default:
        return hipErrorInvalidValue;
    }
  });
  return hipGetLastError();
}

template int default_lines<float>(int, int);
template int default_lines<double>(int, int);
template size_t pass_lds<float>(int, int, int, int);
template size_t pass_lds<double>(int, int, int, int);
template int pass_row_stride<float>(int, int, int);
template int pass_row_stride<double>(int, int, int);
// Every transform kernel may use up to kMaxLDS bytes of dynamic LDS (the gfx950 limit
// per workgroup); set once per process, before any launch or graph capture.
template <typename T, int L> static hipError_t allow_lds_fwd() {
  const void* f[] = {(const void*)&k_fft_x_fwd<T, L>, (const void*)&k_fft_y_fwd<T, L>,
                     (const void*)&k_fft_z_conv<T, L, 1>, (const void*)&k_fft_z_conv<T, L, 2>,
                     (const void*)&k_fft_y_inv<T, L, 3>,
                     (const void*)&k_fft_y_inv<T, L, 4>, (const void*)&k_fft_x_inv<T, L>};
  for (const void* k : f) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLDS);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t allow_lds_forward() {
  hipError_t e = hipSuccess;
#define APM_ALLOW(LL)                                                         \
  if (e == hipSuccess) e = allow_lds_fwd<float, LL>();                         \
  if (e == hipSuccess) e = allow_lds_fwd<double, LL>();
  APM_ALLOW(16) APM_ALLOW(32) APM_ALLOW(64) APM_ALLOW(128) APM_ALLOW(256) APM_ALLOW(512)
  APM_ALLOW(1024)
#undef APM_ALLOW
  return e;
}

template hipError_t launch_pass<float>(int, int, int, int, const ConvJob*, int, int64_t,
                                       const LevelPtrs<float>&, C2<float>*, C2<float>*,
                                       C2<float>*, const void*, hipStream_t);
template hipError_t launch_pass<double>(int, int, int, int, const ConvJob*, int, int64_t,
                                        const LevelPtrs<double>&, C2<double>*, C2<double>*,
                                        C2<double>*, const void*, hipStream_t);

// ---------------------------------------------------------- kernel-table copies --
// One thread per natural-order entry; padding columns (kx >= Mx/2 + 1) are never read.
template <typename T, int KS>
__global__ void k_table_tiles(const double* __restrict__ pairs, T* __restrict__ out, int Mx,
                              int My, int Mz, int comp, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int W = Mx / 2 + 1, Oy = My / 2 + 1;
  const int kx = (int)(i % W);
  const int64_t r = i / W;
  const int ky = (int)(r % Oy), kz = (int)(r / Oy);
  const int64_t o = oct_col(kx, ky, Mx, Mz) + (int64_t)kz * kOctKx;
  if constexpr (KS == 1) {
    out[o] = (T)pairs[2 * i + comp];
  } else {
    out[2 * o] = (T)pairs[2 * i];
    out[2 * o + 1] = (T)pairs[2 * i + 1];
  }
}

template <typename T, int KS>
hipError_t launch_table_tiles(const double* pairs, T* out, int Mx, int My, int Mz, int comp,
                              hipStream_t s) {
  const int64_t n = (int64_t)(Mx / 2 + 1) * (My / 2 + 1) * (Mz / 2 + 1);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_table_tiles<T, KS>), dim3((unsigned)((n + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, pairs, out, Mx, My, Mz, comp, n);
  return hipGetLastError();
}
template hipError_t launch_table_tiles<float, 1>(const double*, float*, int, int, int, int, hipStream_t);
template hipError_t launch_table_tiles<float, 2>(const double*, float*, int, int, int, int, hipStream_t);
template hipError_t launch_table_tiles<double, 1>(const double*, double*, int, int, int, int,
                                                  hipStream_t);
template hipError_t launch_table_tiles<double, 2>(const double*, double*, int, int, int, int,
                                                  hipStream_t);

}  // namespace apm
