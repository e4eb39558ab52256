// Transform passes of the per-grid convolution (Sec. 2.2, Eq. 2): a real 3-D FFT of
// the zero-padded GMF, multiplication by the influence functions with Fourier-space
// differencing, and the inverse transforms of the four outputs (a_x, a_y, a_z, Phi).
//
// Spectrum layout (complex, x fastest): planes z, rows y (My of them), columns
// kx in [0, W), W = Mx/2 + 1.  Five passes per grid:
//   x_fwd   GMF rows (gx reals, zero-padded to Mx) -> half spectra, two real rows
//           per complex FFT                                   (gy*gz rows)
//   y_fwd   columns along y: gy inputs -> My outputs, in place (gz planes)
//   z_conv  columns along z: gz inputs -> Mz-point forward FFT -> times the four
//           multipliers -> four inverse FFTs -> fz outputs each (My*W columns)
//   y_inv   columns along y: My inputs -> fy outputs, in place (4 fz planes)
//   x_inv   two rows of one component per complex inverse FFT, Hermitian rows ->
//           real field-box rows, written as 4-vectors per cell (fy*fz rows)
// Zero planes/rows of the padding are never read or transformed twice: y_fwd reads
// only gy rows, z_conv only gz planes, and the inverse passes write only the field
// box.  Unnormalised transforms; 1/(Mx My Mz) is folded into the kernel table.
#include "apm_kernels.hpp"
#include "device_common.hpp"

namespace apm {

// ------------------------------------------------------------------ x forward --
template <typename T, int L>
__global__ void __launch_bounds__((FFTShape<T, L>::NT))
k_fft_x_fwd(const T* __restrict__ gmf, int gx, int gy, int gz, C2<T>* __restrict__ spec,
            int My, int W, const C2<T>* __restrict__ tw) {
  using S = FFTShape<T, L>;
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int t = threadIdx.x;
  const int b = t / (L / 8), w = t % (L / 8);
  C2<T>* line = lds + b * S::LS;
  const int64_t rows = (int64_t)gy * gz;
  const int64_t q = (int64_t)blockIdx.x * S::NL + b;
  const int64_t ra = 2 * q, rb = 2 * q + 1;
  for (int i = w; i < L; i += L / 8) {
    T xa = 0, xb = 0;
    if (i < gx) {
      if (ra < rows) xa = gmf[ra * gx + i];
      if (rb < rows) xb = gmf[rb * gx + i];
    }
    line[i] = mk<T>(xa, xb);
  }
  __syncthreads();
  fft_line<T, L, false>(line, w, tw);
  if (ra < rows) {
    const int64_t za = ra / gy, ya = ra % gy, zb = rb / gy, yb = rb % gy;
    C2<T>* outa = spec + (za * My + ya) * W;
    C2<T>* outb = spec + (zb * My + yb) * W;
    const T h = (T)0.5;
    for (int k = w; k <= L / 2; k += L / 8) {
      C2<T> z = line[k], m = line[(L - k) & (L - 1)];
      outa[k] = mk<T>(h * (z.x + m.x), h * (z.y - m.y));
      if (rb < rows) outb[k] = mk<T>(h * (z.y + m.y), h * (m.x - z.x));
    }
  }
}

// ------------------------------------------------- strided columns (y passes) --
// Lines along the row index of planes: element (plane p, row r, column c) at
// buf[p * plane_stride + r * W + c].  Reads rows [0, n_in) (rest zero), writes rows
// j in [0, n_out) from transform index (out_off + j) mod L.  In place.
template <typename T, int L, bool INV>
__global__ void __launch_bounds__((FFTShape<T, L>::NT))
k_fft_cols(C2<T>* __restrict__ buf, int64_t plane_stride, int W, int nbw, int n_in, int n_out,
           int out_off, const C2<T>* __restrict__ tw) {
  using S = FFTShape<T, L>;
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int t = threadIdx.x;
  const int64_t p = blockIdx.x / nbw;
  const int c0 = (blockIdx.x % nbw) * S::NL;
  C2<T>* base = buf + p * plane_stride + c0;
  for (int idx = t; idx < S::NL * L; idx += S::NT) {
    const int bb = idx % S::NL, r = idx / S::NL;
    C2<T> v = mk<T>(0, 0);
    if (r < n_in && c0 + bb < W) v = base[(int64_t)r * W + bb];
    lds[bb * S::LS + r] = v;
  }
  __syncthreads();
  const int b = t / (L / 8), w = t % (L / 8);
  fft_line<T, L, INV>(lds + b * S::LS, w, tw);
  __syncthreads();                                   // stores use another mapping
  for (int idx = t; idx < S::NL * n_out; idx += S::NT) {
    const int bb = idx % S::NL, j = idx / S::NL;
    if (c0 + bb < W) base[(int64_t)j * W + bb] = lds[bb * S::LS + ((out_off + j) & (L - 1))];
  }
}

// --------------------------------------------------------- z pass + multiply --
// For one (ky, block of kx): forward FFT along z of gz nonzero planes, then for
// each output component c the product with its multiplier and an inverse FFT:
//   c = 0,1,2: -i d_c(k) Gf(k)   (Fourier-space differencing of the potential)
//   c = 3:      Gp(k)
// kern: octant table of (Gf, Gp), index ((|kz| Oy) + |ky|) W + kx, already scaled.
template <typename T, int L>
__global__ void __launch_bounds__((FFTShape<T, L>::NT))
k_fft_z_conv(const C2<T>* __restrict__ spec, C2<T>* __restrict__ out, int gz, int My, int W,
             int nbw, int fz, int oz, const C2<T>* __restrict__ kern, const T* __restrict__ dxs,
             const T* __restrict__ dys, const T* __restrict__ dzs, const C2<T>* __restrict__ tw) {
  using S = FFTShape<T, L>;
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int t = threadIdx.x;
  const int ky = blockIdx.x / nbw;
  const int c0 = (blockIdx.x % nbw) * S::NL;
  const int64_t pstride = (int64_t)My * W;
  for (int idx = t; idx < S::NL * L; idx += S::NT) {
    const int bb = idx % S::NL, z = idx / S::NL;
    C2<T> v = mk<T>(0, 0);
    if (z < gz && c0 + bb < W) v = spec[z * pstride + (int64_t)ky * W + c0 + bb];
    lds[bb * S::LS + z] = v;
  }
  __syncthreads();
  const int b = t / (L / 8), w = t % (L / 8);
  C2<T>* line = lds + b * S::LS;
  fft_line<T, L, false>(line, w, tw);

  const int kx = c0 + b;
  const bool live = kx < W;
  const int kxc = live ? kx : 0;
  const int Oy = My / 2 + 1;
  const int kyo = ky <= My / 2 ? ky : My - ky;
  const T dxk = dxs[kxc], dyk = dys[ky];
  C2<T> X[8], Gk[8];
  T dzk[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kz = w + q * (L / 8);
    const int kzo = kz <= L / 2 ? kz : L - kz;
    X[q] = line[kz];
    Gk[q] = kern[((int64_t)kzo * Oy + kyo) * W + kxc];
    dzk[q] = dzs[kz];
  }
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kz = w + q * (L / 8);
      C2<T> v;
      if (c == 3) {
        v = mk<T>(Gk[q].y * X[q].x, Gk[q].y * X[q].y);
      } else {
        const T d = (c == 0 ? dxk : (c == 1 ? dyk : dzk[q])) * Gk[q].x;
        v = mk<T>(d * X[q].y, -d * X[q].x);          // -i d G X
      }
      line[kz] = v;
    }
    __syncthreads();
    fft_line<T, L, true>(line, w, tw);
    __syncthreads();                                 // stores use another mapping
    for (int idx = t; idx < S::NL * fz; idx += S::NT) {
      const int bb = idx % S::NL, j = idx / S::NL;
      if (c0 + bb < W)
        out[((int64_t)(c * fz + j) * My + ky) * W + c0 + bb] = lds[bb * S::LS + ((oz + j) & (L - 1))];
    }
    __syncthreads();
  }
  (void)live;
}

// ------------------------------------------------------------------ x inverse --
// Flattened output rows r = j fy + y (j < fz, y < fy) are taken in pairs (2q, 2q+1);
// each component c of a pair is one complex line A_c(row 2q) + i A_c(row 2q+1) with
// Hermitian completion, so the real and imaginary parts of the inverse FFT are the
// two rows.  Pairing rows of the same component keeps magnitudes alike (an
// acceleration and the potential can differ by 1/dx, and a shared complex FFT would
// hand the larger one's rounding to the smaller).  4 lines per row pair; writes
// field[r fx + x] = (a_x, a_y, a_z, Phi).  Rows are contiguous, so no LDS padding.
template <typename T, int L> struct XInvShape {
  static constexpr int NL = FFTShape<T, L>::NL < 4 ? 4 : FFTShape<T, L>::NL;
  static constexpr int NT = NL * (L / 8);
  static constexpr int LS = L;
};

template <typename T, int L>
__global__ void __launch_bounds__((XInvShape<T, L>::NT))
k_fft_x_inv(const C2<T>* __restrict__ out, int fz, int fy, int fx, int My, int W, int ox,
            V4<T>* __restrict__ field, const C2<T>* __restrict__ tw) {
  using S = XInvShape<T, L>;
  constexpr int G = S::NL / 4;
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int t = threadIdx.x;
  const int b = t / (L / 8), w = t % (L / 8);
  const int64_t rows = (int64_t)fz * fy;
  const int64_t q = (int64_t)blockIdx.x * G + b / 4;
  const int c = b & 3;
  const int64_t ra = 2 * q, rb = 2 * q + 1;
  C2<T>* line = lds + b * S::LS;
  if (ra < rows) {
    const C2<T>* A = out + ((int64_t)(c * fz + ra / fy) * My + ra % fy) * W;
    const bool hb = rb < rows;
    const C2<T>* B = out + ((int64_t)(c * fz + (hb ? rb : ra) / fy) * My + (hb ? rb : ra) % fy) * W;
    for (int i = w; i < L; i += L / 8) {
      const int k = i <= L / 2 ? i : L - i;
      C2<T> a = A[k], bq = hb ? B[k] : mk<T>(0, 0);
      if (k == 0 || k == L / 2) { a.y = 0; bq.y = 0; }
      line[i] = i <= L / 2 ? mk<T>(a.x - bq.y, a.y + bq.x) : mk<T>(a.x + bq.y, bq.x - a.y);
    }
  } else {
    for (int i = w; i < L; i += L / 8) line[i] = mk<T>(0, 0);
  }
  __syncthreads();
  fft_line<T, L, true>(line, w, tw);
  __syncthreads();                                   // stores read four lines
  for (int idx = t; idx < G * 2 * fx; idx += S::NT) {
    const int gg = idx / (2 * fx), rem = idx % (2 * fx);
    const int half = rem / fx, x = rem % fx;
    const int64_t r = 2 * ((int64_t)blockIdx.x * G + gg) + half;
    if (r < rows) {
      const int xi = (ox + x) & (L - 1);
      const C2<T>* L0 = lds + (4 * gg) * S::LS + xi;
      V4<T> o;
      if (half == 0) {
        o.x = L0[0].x; o.y = L0[S::LS].x; o.z = L0[2 * S::LS].x; o.w = L0[3 * S::LS].x;
      } else {
        o.x = L0[0].y; o.y = L0[S::LS].y; o.z = L0[2 * S::LS].y; o.w = L0[3 * S::LS].y;
      }
      field[r * fx + x] = o;
    }
  }
}

// ------------------------------------------------------------------ launchers --
template <typename T, int L>
static size_t lds_bytes() { return (size_t)FFTShape<T, L>::NL * FFTShape<T, L>::LS * sizeof(C2<T>); }

#define APM_FFT_DISPATCH(Lv, ...)          \
  switch (Lv) {                            \
    case 16: { constexpr int LL = 16; __VA_ARGS__; } break;   \
    case 32: { constexpr int LL = 32; __VA_ARGS__; } break;   \
    case 64: { constexpr int LL = 64; __VA_ARGS__; } break;   \
    case 128: { constexpr int LL = 128; __VA_ARGS__; } break; \
    case 256: { constexpr int LL = 256; __VA_ARGS__; } break; \
    case 512: { constexpr int LL = 512; __VA_ARGS__; } break; \
    case 1024: { constexpr int LL = 1024; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;  \
  }

template <typename T>
hipError_t launch_grid_convolution(const GridConv<T>& j, hipStream_t s, const LaunchHook& hook) {
  const int W = j.M[0] / 2 + 1;
  const int My = j.M[1];
  // x forward
  hook("fft_x_fwd", 0);
  APM_FFT_DISPATCH(j.M[0], {
    using S = FFTShape<T, LL>;
    const size_t shm = lds_bytes<T, LL>();
    const int64_t pairs = ((int64_t)j.g[1] * j.g[2] + 1) / 2;
    const unsigned nb = (unsigned)((pairs + S::NL - 1) / S::NL);
    hipLaunchKernelGGL((k_fft_x_fwd<T, LL>), dim3(nb), dim3(S::NT), shm, s,
                       j.gmf, j.g[0], j.g[1], j.g[2], j.spec, My, W, (const C2<T>*)j.tw[0]);
  });
  hook("fft_x_fwd", 1);
  // y forward, in place over gz planes
  hook("fft_y_fwd", 0);
  APM_FFT_DISPATCH(j.M[1], {
    using S = FFTShape<T, LL>;
    const size_t shm = lds_bytes<T, LL>();
    const int nbw = (W + S::NL - 1) / S::NL;
    hipLaunchKernelGGL((k_fft_cols<T, LL, false>), dim3((unsigned)(nbw * j.g[2])), dim3(S::NT),
                       shm, s, j.spec, (int64_t)My * W, W, nbw, j.g[1], My, 0,
                       (const C2<T>*)j.tw[1]);
  });
  hook("fft_y_fwd", 1);
  // z pass with multiply, 4 outputs
  hook("fft_z_conv", 0);
  APM_FFT_DISPATCH(j.M[2], {
    using S = FFTShape<T, LL>;
    const size_t shm = lds_bytes<T, LL>();
    const int nbw = (W + S::NL - 1) / S::NL;
    hipLaunchKernelGGL((k_fft_z_conv<T, LL>), dim3((unsigned)(nbw * My)), dim3(S::NT),
                       shm, s, (const C2<T>*)j.spec, j.out, j.g[2], My, W, nbw,
                       j.f[2], j.off[2], (const C2<T>*)j.kern, j.dsym[0], j.dsym[1], j.dsym[2],
                       (const C2<T>*)j.tw[2]);
  });
  hook("fft_z_conv", 1);
  // y inverse over 4 fz planes
  hook("fft_y_inv", 0);
  APM_FFT_DISPATCH(j.M[1], {
    using S = FFTShape<T, LL>;
    const size_t shm = lds_bytes<T, LL>();
    const int nbw = (W + S::NL - 1) / S::NL;
    hipLaunchKernelGGL((k_fft_cols<T, LL, true>), dim3((unsigned)(nbw * 4 * j.f[2])),
                       dim3(S::NT), shm, s, j.out, (int64_t)My * W, W, nbw, My,
                       j.f[1], j.off[1], (const C2<T>*)j.tw[1]);
  });
  hook("fft_y_inv", 1);
  // x inverse into the field box
  hook("fft_x_inv", 0);
  APM_FFT_DISPATCH(j.M[0], {
    using S = XInvShape<T, LL>;
    const size_t shm = (size_t)S::NL * S::LS * sizeof(C2<T>);
    const int64_t pairs = ((int64_t)j.f[1] * j.f[2] + 1) / 2;
    const unsigned nb = (unsigned)((pairs + S::NL / 4 - 1) / (S::NL / 4));
    hipLaunchKernelGGL((k_fft_x_inv<T, LL>), dim3(nb), dim3(S::NT), shm, s,
                       (const C2<T>*)j.out, j.f[2], j.f[1], j.f[0], My, W, j.off[0],
                       (V4<T>*)j.field, (const C2<T>*)j.tw[0]);
  });
  hook("fft_x_inv", 1);
  return hipGetLastError();
}

template hipError_t launch_grid_convolution<float>(const GridConv<float>&, hipStream_t,
                                                   const LaunchHook&);
template hipError_t launch_grid_convolution<double>(const GridConv<double>&, hipStream_t,
                                                    const LaunchHook&);

}  // namespace apm
