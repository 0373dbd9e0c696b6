// Fourier stages of the MW transforms (the O(L^2 log L) part):
//   phi stage   : one workgroup per ring t, DFT of length N1 = 2L-1 along phi
//   theta stage : one workgroup per order m, periodic extension in theta,
//                 DFT of length N1 with the half-sample twiddle, and (forward)
//                 the weight convolution done as a product on an N2-point grid.
// Every DFT of the odd length N1 is evaluated with Bluestein's chirp identity
// on a power-of-two FFT of length N2 >= 4L-3 (the same N2 that the weight
// convolution needs), held entirely in LDS.
#include "mw_internal.h"

namespace mw {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by DIR * i
template <int DIR>
__device__ __forceinline__ double2 mul_dir_i(double2 a)
{
    return DIR < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// Block-wide in-place FFT of length N = 2^logN in LDS (Stockham indexing,
// radix-4 stages preceded by one radix-2 stage when logN is odd; each stage
// reads into registers, synchronises, writes).  Requires blockDim.x >= N/8.
//   DIR = -1:  X_j = sum_k x_k exp(-2 pi i j k / N)
//   DIR = +1:  X_j = sum_k x_k exp(+2 pi i j k / N)   (no 1/N)
// tw[e] = exp(-2 pi i e / N2) of the plan; N divides N2 = N here.
template <int DIR>
__device__ void block_fft(double2* x, int N, int logN, const double2* __restrict__ tw)
{
    const int T = blockDim.x, tid = threadIdx.x;
    int p = 1, logp = 0;
    __syncthreads();
    if (logN & 1) {
        const int NB = N >> 1;
        double2 u[4][2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int i = tid + q * T;
            if (i < NB) { u[q][0] = x[i]; u[q][1] = x[i + NB]; }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int i = tid + q * T;
            if (i < NB) {
                x[2 * i] = cadd(u[q][0], u[q][1]);
                x[2 * i + 1] = csub(u[q][0], u[q][1]);
            }
        }
        p = 2; logp = 1;
        __syncthreads();
    }
    const int NB = N >> 2;
    while (p < N) {
        double2 u[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int i = tid + q * T;
            if (i < NB) {
#pragma unroll
                for (int t = 0; t < 4; ++t) u[q][t] = x[i + t * NB];
            }
        }
        __syncthreads();
        const int sh = logN - logp - 2;  // log2(N / (4p))
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int i = tid + q * T;
            if (i < NB) {
                const int k = i & (p - 1);
#pragma unroll
                for (int t = 1; t < 4; ++t) {
                    double2 w = tw[(t * k) << sh];
                    if (DIR > 0) w = cconj(w);
                    u[q][t] = cmul(u[q][t], w);
                }
                double2 a0 = cadd(u[q][0], u[q][2]);
                double2 a1 = csub(u[q][0], u[q][2]);
                double2 a2 = cadd(u[q][1], u[q][3]);
                double2 a3 = mul_dir_i<DIR>(csub(u[q][1], u[q][3]));
                const int j = ((i - k) << 2) + k;
                x[j] = cadd(a0, a2);
                x[j + p] = cadd(a1, a3);
                x[j + 2 * p] = csub(a0, a2);
                x[j + 3 * p] = csub(a1, a3);
            }
        }
        p <<= 2; logp += 2;
        __syncthreads();
    }
}

// Bluestein DFT of length N1 of the chirped, zero-padded sequence already in
// x[0..N2): on return x[k] * chirp[k] = sum_j a_j exp(-2 pi i j k / N1), k < N1.
__device__ void bluestein_core(double2* x, const Plan& p)
{
    block_fft<-1>(x, p.N2, p.logN2, p.tw);
    for (int j = threadIdx.x; j < p.N2; j += blockDim.x) x[j] = cmul(x[j], p.bhat[j]);
    block_fft<+1>(x, p.N2, p.logN2, p.tw);
}

// XCD-aware column index: consecutive workgroups are dealt round-robin over the
// 8 XCDs; give each XCD a contiguous range of columns so neighbouring columns
// (which share cache lines of the row-major intermediates) meet in one L2.
__device__ __forceinline__ int xcd_column(int ncol)
{
    const int per = (ncol + 7) >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// Forward phi stage (Sec. IV-D): G_m(theta_t) = 2pi/N1 sum_p f(t, p) e^{-i m phi_p}.
// Output G[t][m + L-1].
template <int REAL>
__global__ void k_phi_forward(Plan p, const void* __restrict__ map, double2* __restrict__ G)
{
    extern __shared__ double2 A[];
    const int t = blockIdx.x, L = p.L, N1 = p.N1;
    for (int j = threadIdx.x; j < p.N2; j += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (j < N1) {
            double2 f = REAL ? make_double2(((const double*)map)[(size_t)t * N1 + j], 0.0)
                             : ((const double2*)map)[(size_t)t * N1 + j];
            v = cmul(f, p.chirp[j]);
        }
        A[j] = v;
    }
    bluestein_core(A, p);
    const double sc = 2.0 * 3.14159265358979323846 / (double)N1;
    for (int k = threadIdx.x; k < N1; k += blockDim.x) {
        const int m = (k <= L - 1) ? k : k - N1;
        G[(size_t)t * N1 + (m + L - 1)] = cscale(cmul(A[k], p.chirp[k]), sc);
    }
}

// Forward theta stage for order m (Sec. IV-B..IV-D):
//   extension  Gext(theta_t) = (-1)^{m+s} G_m(theta_{2L-2-t}) for t >= L,
//   F_{m m'} = 1/(2 pi N1) sum_t Gext(theta_t) e^{-i m' theta_t},
//   G_{m m'} = 2 pi sum_{m''} F_{m m''} w(m'' - m')  (product on the N2 grid),
//   fold     H_{m,0} = G_{m,0},  H_{m,n} = G_{m,n} + (-1)^{m+s} G_{m,-n}  (Eq.(Fmm_sym1)).
// Output: Hp records (see mw_internal.h); order m writes its slot of row |m|,
// including the zero pad entry n = L when L is odd.
__global__ void k_theta_forward(Plan p, int s, const double2* __restrict__ G, double* __restrict__ Hp)
{
    extern __shared__ double2 A[];
    const int L = p.L, N1 = p.N1, N2 = p.N2;
    const int mi = xcd_column(N1);
    if (mi >= N1) return;
    const int m = mi - (L - 1);
    const double sig = ((m + s) & 1) ? -1.0 : 1.0;
    for (int j = threadIdx.x; j < N2; j += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (j < N1) {
            double2 g = (j < L) ? G[(size_t)j * N1 + mi] : cscale(G[(size_t)(2 * L - 2 - j) * N1 + mi], sig);
            v = cmul(g, p.chirp[j]);
        }
        A[j] = v;
    }
    bluestein_core(A, p);
    // F_{m'} into registers (N1 <= 8 * blockDim.x), then scatter to slot m' mod N2.
    double2 r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        if (k < N1) r[q] = cmul(cmul(A[k], p.chirp[k]), p.thtw[k]);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N2; j += blockDim.x) A[j] = make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        if (k < N1) {
            const int mp = (k <= L - 1) ? k : k - N1;
            A[(mp + N2) & (N2 - 1)] = r[q];
        }
    }
    block_fft<+1>(A, N2, p.logN2, p.tw);
    for (int j = threadIdx.x; j < N2; j += blockDim.x) A[j] = cmul(A[j], p.what[j]);
    block_fft<-1>(A, N2, p.logN2, p.tw);
    const int am = m < 0 ? -m : m;
    for (int n = threadIdx.x; n < p.Lp; n += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (n < L) {
            v = A[n];
            if (n > 0) v = cadd(v, cscale(A[N2 - n], sig));
        }
        double* rec = Hp + ((size_t)am * p.Lp + n) * 4;
        if (m >= 0) { rec[0] = v.x; rec[1] = v.y; }
        if (m <= 0) { rec[2] = v.x; rec[3] = v.y; }
    }
}

// Inverse theta stage for order m (Sec. IV-E, Eq.(Fmt)):
//   F_m(theta_t) = sum_{m'} F_{m m'} e^{i m' theta_t}, t < L only,
// from the folded F[m + L-1][n] (n >= 0) with F_{m,-n} = (-1)^{m+s} F_{m,n}.
// Output Ft[t][m + L-1].
__global__ void k_theta_inverse(Plan p, int s, const double2* __restrict__ F, double2* __restrict__ Ft)
{
    extern __shared__ double2 A[];
    const int L = p.L, N1 = p.N1, N2 = p.N2;
    const int mi = xcd_column(N1);
    if (mi >= N1) return;
    const int m = mi - (L - 1);
    const double sig = ((m + s) & 1) ? -1.0 : 1.0;
    const double unscale = 2.0 * 3.14159265358979323846 * (double)N1;
    for (int j = threadIdx.x; j < N2; j += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (j < N1) {
            const int mp = (j <= L - 1) ? j : j - N1;
            double2 f = F[(size_t)mi * L + (mp < 0 ? -mp : mp)];
            if (mp < 0) f = cscale(f, sig);
            // y = f e^{+i m' pi/N1};  conj(thtw) * 2 pi N1 = e^{+i m' pi/N1}
            double2 y = cmul(f, cscale(cconj(p.thtw[j]), unscale));
            v = cmul(cconj(y), p.chirp[j]);
        }
        A[j] = v;
    }
    bluestein_core(A, p);
    for (int t = threadIdx.x; t < L; t += blockDim.x)
        Ft[(size_t)t * N1 + mi] = cconj(cmul(A[t], p.chirp[t]));
}

// Inverse phi stage (Eq.(f_pfft)): f(t, p) = sum_m F_m(theta_t) e^{i m phi_p}.
template <int REAL>
__global__ void k_phi_inverse(Plan p, const double2* __restrict__ Ft, void* __restrict__ map)
{
    extern __shared__ double2 A[];
    const int t = blockIdx.x, L = p.L, N1 = p.N1;
    for (int j = threadIdx.x; j < p.N2; j += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (j < N1) {
            const int m = (j <= L - 1) ? j : j - N1;
            v = cmul(cconj(Ft[(size_t)t * N1 + (m + L - 1)]), p.chirp[j]);
        }
        A[j] = v;
    }
    bluestein_core(A, p);
    for (int k = threadIdx.x; k < N1; k += blockDim.x) {
        double2 out = cconj(cmul(A[k], p.chirp[k]));
        if (REAL) ((double*)map)[(size_t)t * N1 + k] = out.x;
        else ((double2*)map)[(size_t)t * N1 + k] = out;
    }
}

int fft_threads(const Plan& p)
{
    int t = p.N2 / 8;
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return t;
}

template <class K>
hipError_t set_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int xcd_grid(int ncol) { return 8 * ((ncol + 7) >> 3); }

}  // namespace

hipError_t launch_phi_forward(const Plan& p, const void* map, int real, double2* G, hipStream_t st)
{
    const size_t lds = (size_t)p.N2 * sizeof(double2);
    hipError_t e;
    if (real) {
        if ((e = set_lds(k_phi_forward<1>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_forward<1>, dim3(p.L), dim3(fft_threads(p)), lds, st, p, map, G);
    } else {
        if ((e = set_lds(k_phi_forward<0>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_forward<0>, dim3(p.L), dim3(fft_threads(p)), lds, st, p, map, G);
    }
    return hipGetLastError();
}

hipError_t launch_theta_forward(const Plan& p, int s, const double2* G, double* Hp, hipStream_t st)
{
    const size_t lds = (size_t)p.N2 * sizeof(double2);
    hipError_t e;
    if ((e = set_lds(k_theta_forward, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_theta_forward, dim3(xcd_grid(p.N1)), dim3(fft_threads(p)), lds, st, p, s, G, Hp);
    return hipGetLastError();
}

hipError_t launch_theta_inverse(const Plan& p, int s, const double2* F, double2* Ft, hipStream_t st)
{
    const size_t lds = (size_t)p.N2 * sizeof(double2);
    hipError_t e;
    if ((e = set_lds(k_theta_inverse, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_theta_inverse, dim3(xcd_grid(p.N1)), dim3(fft_threads(p)), lds, st, p, s, F, Ft);
    return hipGetLastError();
}

hipError_t launch_phi_inverse(const Plan& p, const double2* Ft, void* map, int real, hipStream_t st)
{
    const size_t lds = (size_t)p.N2 * sizeof(double2);
    hipError_t e;
    if (real) {
        if ((e = set_lds(k_phi_inverse<1>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_inverse<1>, dim3(p.L), dim3(fft_threads(p)), lds, st, p, Ft, map);
    } else {
        if ((e = set_lds(k_phi_inverse<0>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_phi_inverse<0>, dim3(p.L), dim3(fft_threads(p)), lds, st, p, Ft, map);
    }
    return hipGetLastError();
}

}  // namespace mw
