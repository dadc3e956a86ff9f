// Block-mode coarse field, one level: at each cell centre t the field of the
// monopole Q_s and dipole P_s of every cell s outside the B^3 block around
// t, with its first and second gradients (the second-order local expansion
// about t).  With R = (t - s) h and T^n = grad^n (1/r),
//
//   E = -Q T^1 + P.T^2,   J = -Q T^2 + P.T^3,   H = -Q T^3 + P.T^4,
//
// a convolution over the grid: T^n((t - s) h) = h^-(n+1) T^n(t - s), so with
// P' = P / h every term is a fixed kernel of the integer offset d = t - s
// (zero for |d|_inf <= B/2) applied to (Q, P'), scaled by h^-2, h^-3, h^-4.
// Offsets span [-31, 31] for G <= 32, so a 64^3 period holds the linear
// convolution.  Transforms are 64-point FFTs across the 64 lanes of a
// wavefront along x, y and z, with planes and slabs staged in LDS:
//
//   forward:   (Q + i P'x, P'y + i P'z) per cell -> two packed spectra;
//   product:   unpack the four input spectra, 15 output spectra from the
//              30 kernel spectra (T^1, T^3 odd: imaginary; T^2, T^4 even:
//              real), packed in pairs;
//   inverse:   eight packed transforms -> 15 real components per cell.
//
// The kernel spectra depend only on B; they are made once at set-up by the
// same transforms.  FP32 transforms, FP64 kernel values and outputs.
#include "ld_ffconv.h"

#include <cstddef>

namespace {

constexpr int kP = 64;                 // period per axis
constexpr int kPP = kP * kP * kP;
constexpr int kPad = kP + 1;           // LDS row pitch: columns hit distinct banks
constexpr int kNSpec = 30;             // T1 (3), T2 (6), T3 (9), T4 (12) components
constexpr int kNPair = 15;             // set-up: kernel components packed in pairs
constexpr int kNOutPack = 8;           // 15 output components packed in pairs
constexpr int kT = 1024;               // threads of the plane and slab kernels (16 waves)

// Components of T^n = grad^n (1/r) kept, as (rank, axis indices).
struct TComp {
    int n, a[4];
};
__constant__ TComp kTComp[kNSpec] = {
    {1, {0}}, {1, {1}}, {1, {2}},
    {2, {0, 0}}, {2, {0, 1}}, {2, {0, 2}}, {2, {1, 1}}, {2, {1, 2}}, {2, {2, 2}},
    {3, {0, 0, 0}}, {3, {0, 0, 1}}, {3, {0, 0, 2}}, {3, {0, 1, 1}}, {3, {0, 1, 2}},
    {3, {0, 2, 2}}, {3, {1, 1, 1}}, {3, {1, 1, 2}}, {3, {1, 2, 2}},
    {4, {0, 0, 0, 0}}, {4, {0, 0, 0, 1}}, {4, {0, 0, 0, 2}}, {4, {0, 0, 1, 1}},
    {4, {0, 0, 1, 2}}, {4, {0, 0, 2, 2}}, {4, {0, 1, 1, 1}}, {4, {0, 1, 1, 2}},
    {4, {0, 1, 2, 2}}, {4, {1, 1, 1, 1}}, {4, {1, 1, 1, 2}}, {4, {1, 1, 2, 2}},
};

__device__ __forceinline__ int rev6(int l) { return (int)(__builtin_bitreverse32((unsigned)l) >> 26); }

// w[k] = exp(-2 pi i k / 64), k < 32, from FP64 sines.
__device__ __forceinline__ void make_twiddles(float2* tw) {
    for (int k = threadIdx.x; k < 32; k += blockDim.x) {
        double s, c;
        sincospi(k / 32.0, &s, &c);
        tw[k] = make_float2((float)c, (float)-s);
    }
}

// 64-point DFT across a wavefront by decimation in frequency: lane l holds
// x[l] on entry and X[rev6(l)] on exit; INV conjugates the twiddles (no 1/64).
template <bool INV>
__device__ __forceinline__ float2 fft64(float2 v, int lane, const float2* tw) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const float px = __shfl_xor(v.x, m), py = __shfl_xor(v.y, m);
        if (lane & m) {
            const float2 w = tw[(lane & (m - 1)) * (32 / m)];
            const float wy = INV ? -w.y : w.y;
            const float dx = px - v.x, dy = py - v.y;    // (partner - own) w
            v = make_float2(dx * w.x - dy * wy, dx * wy + dy * w.x);
        } else {
            v = make_float2(v.x + px, v.y + py);
        }
    }
    return v;
}

// Forward transform along x then y of plane z = blockIdx.x of array
// blockIdx.y.  MOM: the plane is built from the cell moments (array 0:
// Q + i P'x, array 1: P'y + i P'z; zero outside the G^2 corner) and only its
// first G rows are transformed along x; otherwise it is read from src (may
// be dst: each workgroup reads its whole plane before writing it).
template <bool MOM>
__global__ __launch_bounds__(kT) void k_conv_fwd_xy(const double* __restrict__ mom, int G,
                                                    const double* __restrict__ hp,
                                                    const float2* src, float2* dst) {
    __shared__ float2 pl[kP * kPad];
    __shared__ float2 tw[32];
    make_twiddles(tw);
    const int z = blockIdx.x, arr = blockIdx.y;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const size_t plane = ((size_t)arr * kP + z) * kP * kP;
    const double ih = MOM ? 1.0 / *hp : 0.0;
    for (int e = t; e < kP * kP; e += kT) {
        const int y = e >> 6, x = e & 63;
        float2 v = make_float2(0.f, 0.f);
        if (MOM) {
            if (x < G && y < G) {
                const double* m = mom + 4 * (((size_t)z * G + y) * G + x);
                v = arr == 0 ? make_float2((float)m[0], (float)(m[1] * ih))
                             : make_float2((float)(m[2] * ih), (float)(m[3] * ih));
            }
        } else {
            v = src[plane + e];
        }
        pl[y * kPad + x] = v;
    }
    __syncthreads();
    const int rows = MOM ? G : kP;
    for (int y = wv; y < rows; y += kT / 64) {
        const float2 v = fft64<false>(pl[y * kPad + lane], lane, tw);
        pl[y * kPad + rev6(lane)] = v;
    }
    __syncthreads();
    for (int x = wv; x < kP; x += kT / 64) {
        const float2 v = fft64<false>(pl[lane * kPad + x], lane, tw);
        pl[rev6(lane) * kPad + x] = v;
    }
    __syncthreads();
    for (int e = t; e < kP * kP; e += kT) dst[plane + e] = pl[(e >> 6) * kPad + (e & 63)];
}

// Transform along z of slab y = blockIdx.x of array blockIdx.y, in place.
// Forward: planes z >= nz are zero (not read).  Inverse: only planes z < nz
// of the result are written.
template <bool INV>
__global__ __launch_bounds__(kT) void k_conv_z(float2* buf, int nz) {
    __shared__ float2 sl[kP * kPad];   // [z][x]
    __shared__ float2 tw[32];
    make_twiddles(tw);
    const int y = blockIdx.x;
    float2* a = buf + (size_t)blockIdx.y * kPP;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int e = t; e < kP * kP; e += kT) {
        const int z = e >> 6, x = e & 63;
        sl[z * kPad + x] = (INV || z < nz) ? a[((size_t)z * kP + y) * kP + x]
                                           : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int x = wv; x < kP; x += kT / 64) {
        const float2 v = fft64<INV>(sl[lane * kPad + x], lane, tw);
        sl[rev6(lane) * kPad + x] = v;
    }
    __syncthreads();
    const int zout = INV ? nz : kP;
    for (int e = t; e < zout * kP; e += kT) {
        const int z = e >> 6, x = e & 63;
        a[((size_t)z * kP + y) * kP + x] = sl[z * kPad + x];
    }
}

// Spectrum at -k of the same array.
__device__ __forceinline__ int neg_index(int k) {
    const int kx = k & 63, ky = (k >> 6) & 63, kz = k >> 12;
    return ((((kP - kz) & 63) * kP + ((kP - ky) & 63)) * kP) + ((kP - kx) & 63);
}

// From Z = F(a + i b), a and b real: F(a) = (Z + conj Z_-) / 2 and
// F(b) = -i (Z - conj Z_-) / 2 with Z_- = Z(-k).
__device__ __forceinline__ float2 unpack_re(float2 z, float2 zm) {
    return make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
}
__device__ __forceinline__ float2 unpack_im(float2 z, float2 zm) {
    return make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
}

// Per frequency: the 15 output spectra from the input spectra and the
// kernel spectra s (K^n = i s for odd n, s for even n), packed in pairs.
__global__ __launch_bounds__(256) void k_conv_mul(const float2* __restrict__ in,
                                                  const float* __restrict__ spec,
                                                  float2* __restrict__ out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= kPP) return;
    const int km = neg_index(k);
    const float2 z1 = in[k], z1m = in[km], z2 = in[kPP + k], z2m = in[kPP + km];
    const float2 Q = unpack_re(z1, z1m), Px = unpack_im(z1, z1m);
    const float2 Py = unpack_re(z2, z2m), Pz = unpack_im(z2, z2m);
    float s[kNSpec];
#pragma unroll
    for (int c = 0; c < kNSpec; ++c) s[c] = spec[(size_t)c * kPP + k];
    // P . (real kernel row a, b, c)
    auto pdot = [&](float a, float b, float c) {
        return make_float2(Px.x * a + Py.x * b + Pz.x * c, Px.y * a + Py.y * b + Pz.y * c);
    };
    float2 o[16];
    // E_a = -Q (i s1_a) + sum_b P_b s2_ab
    {
        const float2 p0 = pdot(s[3], s[4], s[5]), p1 = pdot(s[4], s[6], s[7]),
                     p2 = pdot(s[5], s[7], s[8]);
        o[0] = make_float2(p0.x + s[0] * Q.y, p0.y - s[0] * Q.x);
        o[1] = make_float2(p1.x + s[1] * Q.y, p1.y - s[1] * Q.x);
        o[2] = make_float2(p2.x + s[2] * Q.y, p2.y - s[2] * Q.x);
    }
    // J_ab = -Q s2_ab + i sum_c P_c s3_abc
    {
        const float2 u[5] = {pdot(s[9], s[10], s[11]), pdot(s[10], s[12], s[13]),
                             pdot(s[11], s[13], s[14]), pdot(s[12], s[15], s[16]),
                             pdot(s[13], s[16], s[17])};
        const float s2[5] = {s[3], s[4], s[5], s[6], s[7]};
#pragma unroll
        for (int q = 0; q < 5; ++q)
            o[3 + q] = make_float2(-s2[q] * Q.x - u[q].y, -s2[q] * Q.y + u[q].x);
    }
    // H_abc = -Q (i s3_abc) + sum_d P_d s4_abcd
    {
        const float2 u[7] = {pdot(s[18], s[19], s[20]), pdot(s[19], s[21], s[22]),
                             pdot(s[20], s[22], s[23]), pdot(s[21], s[24], s[25]),
                             pdot(s[22], s[25], s[26]), pdot(s[24], s[27], s[28]),
                             pdot(s[25], s[28], s[29])};
        const float s3[7] = {s[9], s[10], s[11], s[12], s[13], s[15], s[16]};
#pragma unroll
        for (int q = 0; q < 7; ++q)
            o[8 + q] = make_float2(u[q].x + s3[q] * Q.y, u[q].y - s3[q] * Q.x);
    }
    o[15] = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < kNOutPack; ++p) {
        const float2 a = o[2 * p], b = o[2 * p + 1];
        out[(size_t)p * kPP + k] = make_float2(a.x - b.y, a.y + b.x);   // a + i b
    }
}

// Output component of packed slot li (0..14) in the 19-entry cell layout.
__constant__ int kOutComp[15] = {0, 1, 2, 3, 4, 5, 6, 7, 9, 10, 11, 12, 13, 15, 16};

// Inverse transform along y then x of plane z = blockIdx.x (< G) of packed
// output array blockIdx.y; the G^2 corner goes to E with the h powers and
// the 1/64^3 of the inverse.
__global__ __launch_bounds__(kT) void k_conv_inv_xy(const float2* __restrict__ buf, int G,
                                                    const double* __restrict__ hp,
                                                    double* __restrict__ E) {
    __shared__ float2 pl[kP * kPad];
    __shared__ float2 tw[32];
    make_twiddles(tw);
    const int z = blockIdx.x, p = blockIdx.y;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const float2* a = buf + (size_t)p * kPP + (size_t)z * kP * kP;
    for (int e = t; e < kP * kP; e += kT) pl[(e >> 6) * kPad + (e & 63)] = a[e];
    __syncthreads();
    for (int x = wv; x < kP; x += kT / 64) {
        const float2 v = fft64<true>(pl[lane * kPad + x], lane, tw);
        pl[rev6(lane) * kPad + x] = v;
    }
    __syncthreads();
    const double h = *hp, ih = 1.0 / h, norm = 1.0 / ((double)kPP);
    const int la = 2 * p, lb = 2 * p + 1;
    auto scale = [&](int li) {
        return norm * ih * ih * (li < 3 ? 1.0 : (li < 8 ? ih : ih * ih));
    };
    const double sa = scale(la), sb = scale(lb);
    const int ca = kOutComp[la], cb = lb < 15 ? kOutComp[lb] : -1;
    for (int y = wv; y < G; y += kT / 64) {
        const float2 v = fft64<true>(pl[y * kPad + lane], lane, tw);
        const int x = rev6(lane);
        if (x < G) {
            double* o = E + (((size_t)z * G + y) * G + x) * 19;
            o[ca] = sa * (double)v.x;
            if (cb >= 0) o[cb] = sb * (double)v.y;
        }
    }
}

// Set-up: the kernel components at every offset of the period (offset d per
// axis: index i < 32 -> i, i > 32 -> i - 64, i = 32 unused -> 0), zero in
// the block, packed in pairs (component 2p + i component 2p+1).
__global__ __launch_bounds__(256) void k_conv_kernels(int half, float2* __restrict__ out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kPP) return;
    const int ix = e & 63, iy = (e >> 6) & 63, iz = e >> 12;
    auto off = [](int i) { return i < 32 ? i : i - 64; };
    const int dx = off(ix), dy = off(iy), dz = off(iz);
    const bool zero = ix == 32 || iy == 32 || iz == 32 ||
                      (abs(dx) <= half && abs(dy) <= half && abs(dz) <= half);
    const double R[3] = {(double)dx, (double)dy, (double)dz};
    const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double ir = zero ? 0.0 : 1.0 / sqrt(r2), ir2 = ir * ir;
    const double u3 = ir * ir2, u5 = u3 * ir2, u7 = u5 * ir2, u9 = u7 * ir2;
    float v[kNSpec];
    for (int c = 0; c < kNSpec; ++c) {
        const TComp tc = kTComp[c];
        const int* a = tc.a;
        auto d = [&](int i, int j) { return a[i] == a[j] ? 1.0 : 0.0; };
        double val;
        if (tc.n == 1) {
            val = -R[a[0]] * u3;
        } else if (tc.n == 2) {
            val = 3.0 * R[a[0]] * R[a[1]] * u5 - d(0, 1) * u3;
        } else if (tc.n == 3) {
            val = -15.0 * R[a[0]] * R[a[1]] * R[a[2]] * u7 +
                  3.0 * (d(0, 1) * R[a[2]] + d(0, 2) * R[a[1]] + d(1, 2) * R[a[0]]) * u5;
        } else {
            const double Ra = R[a[0]], Rb = R[a[1]], Rc = R[a[2]], Rd = R[a[3]];
            val = 105.0 * Ra * Rb * Rc * Rd * u9 -
                  15.0 * (d(0, 1) * Rc * Rd + d(0, 2) * Rb * Rd + d(0, 3) * Rb * Rc +
                          d(1, 2) * Ra * Rd + d(1, 3) * Ra * Rc + d(2, 3) * Ra * Rb) * u7 +
                  3.0 * (d(0, 1) * d(2, 3) + d(0, 2) * d(1, 3) + d(0, 3) * d(1, 2)) * u5;
        }
        v[c] = (float)val;
    }
    for (int p = 0; p < kNPair; ++p) out[(size_t)p * kPP + e] = make_float2(v[2 * p], v[2 * p + 1]);
}

// Set-up: unpack pair p's spectrum into its two components, keeping the
// imaginary part of odd-rank (T^1, T^3) and the real part of even-rank ones.
__global__ __launch_bounds__(256) void k_conv_spec(const float2* __restrict__ Z,
                                                   float* __restrict__ spec) {
    const int k = blockIdx.x * 256 + threadIdx.x, p = blockIdx.y;
    if (k >= kPP) return;
    const float2 z = Z[(size_t)p * kPP + k], zm = Z[(size_t)p * kPP + neg_index(k)];
    const float2 fa = unpack_re(z, zm), fb = unpack_im(z, zm);
    const int ca = 2 * p, cb = 2 * p + 1;
    auto odd = [](int c) { return c < 3 || (c >= 9 && c < 18); };
    spec[(size_t)ca * kPP + k] = odd(ca) ? fa.y : fa.x;
    spec[(size_t)cb * kPP + k] = odd(cb) ? fb.y : fb.x;
}

}  // namespace

namespace ld {

hipError_t conv_setup(LocalConv* lc, int B, hipStream_t s) {
    conv_free(lc);
    lc->B = B;
    hipError_t e = hipMalloc(&lc->work, sizeof(float2) * (size_t)kNPair * kPP);
    if (e != hipSuccess) return e;
    e = hipMalloc(&lc->spec, sizeof(float) * (size_t)kNSpec * kPP);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_conv_kernels, dim3(kPP / 256), dim3(256), 0, s, B / 2, lc->work);
    hipLaunchKernelGGL(k_conv_fwd_xy<false>, dim3(kP, kNPair), dim3(kT), 0, s, nullptr, 0,
                       nullptr, lc->work, lc->work);
    hipLaunchKernelGGL(k_conv_z<false>, dim3(kP, kNPair), dim3(kT), 0, s, lc->work, kP);
    hipLaunchKernelGGL(k_conv_spec, dim3(kPP / 256, kNPair), dim3(256), 0, s, lc->work, lc->spec);
    return hipGetLastError();
}

hipError_t conv_local(const LocalConv* lc, const double* mom, int G, const double* h, double* E,
                      hipStream_t s) {
    float2* in = lc->work;                 // 2 packed input spectra
    float2* out = lc->work + 2 * (size_t)kPP;   // 8 packed output spectra
    hipLaunchKernelGGL(k_conv_fwd_xy<true>, dim3(G, 2), dim3(kT), 0, s, mom, G, h, nullptr, in);
    hipLaunchKernelGGL(k_conv_z<false>, dim3(kP, 2), dim3(kT), 0, s, in, G);
    hipLaunchKernelGGL(k_conv_mul, dim3(kPP / 256), dim3(256), 0, s, in, lc->spec, out);
    hipLaunchKernelGGL(k_conv_z<true>, dim3(kP, kNOutPack), dim3(kT), 0, s, out, G);
    hipLaunchKernelGGL(k_conv_inv_xy, dim3(G, kNOutPack), dim3(kT), 0, s, out, G, h, E);
    return hipGetLastError();
}

void conv_free(LocalConv* lc) {
    if (lc->work) (void)hipFree(lc->work);
    if (lc->spec) (void)hipFree(lc->spec);
    lc->work = nullptr;
    lc->spec = nullptr;
}

}  // namespace ld
