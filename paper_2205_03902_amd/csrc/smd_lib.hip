// libimsp: sparse matrix decomposition (Algorithm 2) on dense N^2 x N^2 matrices, behind the
// C ABI of include/smd.h.  Dense complex products go to rocBLAS (column-major): a row-major
// product C = op(A) op(B) is the column-major product C^T = op(B)^T op(A)^T, i.e. the same
// operations with the operands swapped.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "ms.h"
#include "smd.h"

namespace {

thread_local std::string s_err;

int32_t sfail(int32_t st, const std::string &msg)
{
    s_err = msg;
    return st;
}

constexpr size_t kAlign = 256;
constexpr size_t kBlasWorkspace = (size_t)32 << 20;
constexpr int kRed = 256;   // reduction partials

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
unsigned blocks(long long n) { return (unsigned)std::min<long long>(65535, (n + 255) / 256); }

// ---------------------------------------------------------------------------------------
// kernels

__global__ void dft_kernel(float2 *F, int n)
{
    const long long n2 = (long long)n * n;
    const double TWO_PI = 6.283185307179586476925286766559;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2 * n2;
         i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i / n2), c = (int)(i - (long long)r * n2);
        const int ky = r / n, kx = r % n, y = c / n, x = c % n;
        const int ph = (ky * y + kx * x) % n;                 // exact integer phase
        double s, co;
        sincos(-TWO_PI * ph / n, &s, &co);
        F[i] = make_float2((float)co, (float)s);
    }
}

// T[r][c] = h(q_r) F[r][c], h = exp(-i pi dz lambda q^2) (eq. fresnel_element, no tilt).
__global__ void h_rows_kernel(const float2 *F, float2 *T, int n, double dz, double lambda, double dx)
{
#pragma clang fp contract(off)
    const long long n2 = (long long)n * n;
    const double PI = 3.14159265358979323846264338327950288;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2 * n2;
         i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i / n2);
        const int ky = r / n, kx = r % n;
        const double qy = (double)(ky < n / 2 ? ky : ky - n) / (n * dx);
        const double qx = (double)(kx < n / 2 ? kx : kx - n) / (n * dx);
        double s, co;
        sincos(-PI * dz * lambda * (qy * qy + qx * qx), &s, &co);
        const float2 f = F[i];
        const double hr = co, hi = s;
        T[i] = make_float2((float)(hr * f.x - hi * f.y), (float)(hr * f.y + hi * f.x));
    }
}

// P[i][s] = probe[(y - py) mod n][(x - px) mod n], i = (y, x).
__global__ void probe_matrix_kernel(const float2 *probe, const int2 *pos, float2 *P, int n, long long S)
{
    const long long n2 = (long long)n * n;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n2 * S;
         t += (long long)gridDim.x * blockDim.x) {
        const long long i = t / S, s = t - i * S;
        const int y = (int)(i / n), x = (int)(i % n);
        const int2 p = pos[s];
        const int yy = ((y - p.x) % n + n) % n, xx = ((x - p.y) % n + n) % n;
        P[t] = probe[yy * n + xx];
    }
}

__global__ void set_diag_kernel(float2 *A, const float2 *d, long long n2, float2 scale)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2 * n2;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i / n2, c = i - r * n2;
        float2 v = make_float2(0.f, 0.f);
        if (r == c) {
            const float2 e = d ? d[r] : make_float2(1.f, 0.f);
            v = make_float2(scale.x * e.x - scale.y * e.y, scale.x * e.y + scale.y * e.x);
        }
        A[i] = v;
    }
}

// out[r][c] = s * d[r] in[r][c] (rows) or s * in[r][c] d[c] (columns).
__global__ void diag_scale_kernel(float2 *out, const float2 *in, const float2 *d, long long n2, int rows, float2 s)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2 * n2;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i / n2, c = i - r * n2;
        const float2 e = d[rows ? r : c], v = in[i];
        const float2 t = make_float2(e.x * v.x - e.y * v.y, e.x * v.y + e.y * v.x);
        out[i] = make_float2(s.x * t.x - s.y * t.y, s.x * t.y + s.y * t.x);
    }
}

// Amplitude residual of Z = F A P against I [S][N^2] (Z is [N^2][S]); FP64 loss partials.
__global__ __launch_bounds__(256) void smd_residual_kernel(float2 *Z, const float *I, long long n2, long long S,
                                                         double *part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n2 * S;
         t += (long long)gridDim.x * blockDim.x) {
        const long long k = t / S, s = t - k * S;
        const float2 z = Z[t];
        const float m = I[s * n2 + k];
        const double a = sqrt((double)z.x * z.x + (double)z.y * z.y);
        const double d = sqrt((double)m) - a;
        acc += d * d;
        const float af = (float)a;
        Z[t] = (af == 0.0f) ? make_float2(0.f, 0.f)
                            : make_float2(z.x - sqrtf(m) * (z.x / af), z.y - sqrtf(m) * (z.y / af));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = 1/2 sum of the partials (fixed order).
__global__ void half_sum_kernel(const double *part, int n, double *out)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = 0.5 * s;
}

// grad[k] = sum_j U[k][j] conj(S[k][j]), FP64 accumulation, one block per k.
__global__ __launch_bounds__(256) void row_dot_conj_kernel(const float2 *U, const float2 *S, long long n2,
                                                         double2 *grad)
{
    __shared__ double re[256], im[256];
    const long long k = blockIdx.x;
    double ar = 0.0, ai = 0.0;
    for (long long j = threadIdx.x; j < n2; j += 256) {
        const float2 u = U[k * n2 + j], s = S[k * n2 + j];
        ar += (double)u.x * s.x + (double)u.y * s.y;
        ai += (double)u.y * s.x - (double)u.x * s.y;
    }
    re[threadIdx.x] = ar;
    im[threadIdx.x] = ai;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            re[threadIdx.x] += re[threadIdx.x + w];
            im[threadIdx.x] += im[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[k] = make_double2(re[0], im[0]);
}

// max |d|^2 of each of M diagonals (one block each).
__global__ __launch_bounds__(256) void peak_kernel(const float2 *d, long long n2, double *peak2)
{
    __shared__ double red[256];
    const float2 *v = d + (long long)blockIdx.x * n2;
    double mx = 0.0;
    for (long long i = threadIdx.x; i < n2; i += 256) mx = fmax(mx, (double)v[i].x * v[i].x + (double)v[i].y * v[i].y);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) peak2[blockIdx.x] = red[0];
}

// o_new = Proj(o - conj(lambda) / c grad), c = |lambda|^2 prod_{m != l} peak2_m; one block.
__global__ __launch_bounds__(256) void prox_update_kernel(const float2 *o, const double2 *grad, const double *peak2,
                                                          int M, int l, double lr, double li, long long n2,
                                                          float2 *out)
{
    __shared__ double red[256];
    double c = lr * lr + li * li;
    for (int m = 0; m < M; ++m)
        if (m != l) c *= peak2[m];
    const double inv = c > 0.0 ? 1.0 / c : 0.0;
    // conj(lambda) grad
    double acc = 0.0;
    for (long long k = threadIdx.x; k < n2; k += 256) {
        const double2 g = grad[k];
        const double tr = lr * g.x + li * g.y, ti = lr * g.y - li * g.x;
        const double nr = (double)o[k].x - inv * tr, ni = (double)o[k].y - inv * ti;
        acc += nr * nr + ni * ni;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double norm = sqrt(red[0]);
    const double sc = norm > 0.0 ? 1.0 / norm : 0.0;
    for (long long k = threadIdx.x; k < n2; k += 256) {
        const double2 g = grad[k];
        const double tr = lr * g.x + li * g.y, ti = lr * g.y - li * g.x;
        out[k] = make_float2((float)(((double)o[k].x - inv * tr) * sc), (float)(((double)o[k].y - inv * ti) * sc));
    }
}

// Partials of Tr(At^H Ah) (re, im) and Tr(At^H At).
__global__ __launch_bounds__(256) void trace_kernel(const float2 *At, const float2 *Ah, long long count, double *part)
{
    __shared__ double r0[256], r1[256], r2[256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const float2 t = At[i], h = Ah[i];
        a += (double)t.x * h.x + (double)t.y * h.y;
        b += (double)t.x * h.y - (double)t.y * h.x;
        c += (double)t.x * t.x + (double)t.y * t.y;
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    r2[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r0[threadIdx.x] += r0[threadIdx.x + w];
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = r0[0];
        part[3 * blockIdx.x + 1] = r1[0];
        part[3 * blockIdx.x + 2] = r2[0];
    }
}

// out = s in (complex scalar s, FP64 product).
__global__ void scale_kernel(float2 *out, const float2 *in, long long count, double sr, double si)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const float2 v = in[i];
        out[i] = make_float2((float)(sr * v.x - si * v.y), (float)(sr * v.y + si * v.x));
    }
}

}  // namespace

struct smd_plan {
    int n = 0, n2 = 0, M = 0;
    long long S = 0;
    double dx = 0, lambda = 0;
    std::vector<double> dz;
    std::vector<int> pos;   // (y, x) pairs
    char *ws = nullptr;
    size_t F, G, P, T1, T2, X, U, Z, R, pfx, sfx, old, grad, peak, part, scal, posd, blas, total;
    rocblas_handle h = nullptr;
    double mu_a = 0.0;
    bool ready = false;

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    size_t mat() const { return (size_t)n2 * n2; }
};

namespace {

void plan_layout(smd_plan &p)
{
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return r;
    };
    const size_t mb = p.mat() * 8, sb = (size_t)p.n2 * p.S * 8;
    p.F = take(mb);
    p.G = take(mb * std::max(p.M - 1, 1));
    p.P = take(sb);
    p.T1 = take(mb);
    p.T2 = take(mb);
    p.X = take(mb);
    p.U = take(mb);
    p.Z = take(sb);
    p.R = take(sb);
    p.pfx = take(mb * p.M);
    p.sfx = take(mb * p.M);
    p.old = take((size_t)p.M * p.n2 * 8);
    p.grad = take((size_t)p.n2 * 16);
    p.peak = take((size_t)p.M * 8);
    p.part = take((size_t)kRed * 3 * 8);
    p.scal = take(64);
    p.posd = take((size_t)p.S * 8);
    p.blas = take(kBlasWorkspace);
    p.total = o;
}

int32_t check_problem(const smd_problem *pb)
{
    if (!pb) return sfail(MS_ERR_INVALID_ARG, "problem is NULL");
    const int n = pb->n;
    if (n != 4 && n != 8 && n != 16 && n != 32 && n != 64)
        return sfail(MS_ERR_INVALID_ARG, "n must be 4, 8, 16, 32 or 64 (dense N^2 x N^2 matrices)");
    if (pb->n_slices < 1 || pb->n_slices > 16) return sfail(MS_ERR_INVALID_ARG, "n_slices must be in [1, 16]");
    if (pb->n_pos < 1 || pb->n_pos > 65536) return sfail(MS_ERR_INVALID_ARG, "n_pos must be in [1, 65536]");
    if (!pb->positions || (pb->n_slices > 1 && !pb->dz)) return sfail(MS_ERR_INVALID_ARG, "positions or dz is NULL");
    for (long long s = 0; s < pb->n_pos; ++s)
        for (int c = 0; c < 2; ++c) {
            const double v = pb->positions[2 * s + c];
            if (!std::isfinite(v) || v != std::floor(v) || std::fabs(v) > 1e6)
                return sfail(MS_ERR_INVALID_ARG, "positions must be integer shifts (full-field model)");
        }
    for (int m = 0; m + 1 < pb->n_slices; ++m)
        if (!std::isfinite(pb->dz[m])) return sfail(MS_ERR_INVALID_ARG, "dz must be finite");
    if (!(pb->pixel_size > 0) || !(pb->wavelength > 0)) return sfail(MS_ERR_INVALID_ARG, "need positive dx, lambda");
    return MS_OK;
}

bool blas_ok(rocblas_status st, const char *what)
{
    if (st == rocblas_status_success) return true;
    s_err = std::string(what) + ": rocBLAS status " + std::to_string((int)st);
    return false;
}

// Row-major C (m x n) = alpha op(A) op(B) + beta C.
bool gemm(smd_plan *p, rocblas_operation opA, rocblas_operation opB, int m, int n, int k, std::complex<float> alpha,
          const float2 *A, int lda, const float2 *B, int ldb, std::complex<float> beta, float2 *C, int ldc)
{
    const rocblas_float_complex al(alpha.real(), alpha.imag()), be(beta.real(), beta.imag());
    return blas_ok(rocblas_cgemm(p->h, opB, opA, n, m, k, &al, reinterpret_cast<const rocblas_float_complex *>(B), ldb,
                                 reinterpret_cast<const rocblas_float_complex *>(A), lda, &be,
                                 reinterpret_cast<rocblas_float_complex *>(C), ldc),
                   "rocblas_cgemm");
}

constexpr rocblas_operation N_ = rocblas_operation_none, H_ = rocblas_operation_conjugate_transpose;

int32_t hip_ok(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return MS_OK;
    return sfail(MS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// A = scale O_M G_{M-1} ... G_1 O_1 into `out`; uses T1.
bool compose_into(smd_plan *p, hipStream_t st, const float2 *sl, std::complex<float> scale, float2 *out)
{
    const long long n2 = p->n2;
    const float2 one = make_float2(1.f, 0.f);
    const float2 sc = make_float2(scale.real(), scale.imag());
    set_diag_kernel<<<blocks(n2 * n2), 256, 0, st>>>(out, sl, n2, p->M == 1 ? sc : one);
    for (int m = 1; m < p->M; ++m) {
        if (!gemm(p, N_, N_, p->n2, p->n2, p->n2, 1.0f, p->at<float2>(p->G) + (size_t)(m - 1) * p->mat(), p->n2, out,
                  p->n2, 0.0f, p->at<float2>(p->T1), p->n2))
            return false;
        diag_scale_kernel<<<blocks(n2 * n2), 256, 0, st>>>(out, p->at<float2>(p->T1), sl + (size_t)m * n2, n2, 1,
                                                           m + 1 == p->M ? sc : one);
    }
    return true;
}

}  // namespace

extern "C" {

int32_t smd_workspace_size(const smd_problem *pb, size_t *ws_bytes)
{
    int32_t s = check_problem(pb);
    if (s != MS_OK) return s;
    if (!ws_bytes) return sfail(MS_ERR_INVALID_ARG, "ws_bytes is NULL");
    smd_plan p;
    p.n = pb->n;
    p.n2 = pb->n * pb->n;
    p.M = pb->n_slices;
    p.S = pb->n_pos;
    plan_layout(p);
    *ws_bytes = p.total;
    return MS_OK;
}

int32_t smd_plan_create(const smd_problem *pb, void *workspace, size_t ws_bytes, smd_plan **out)
{
    int32_t s = check_problem(pb);
    if (s != MS_OK) return s;
    if (!out || !workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
        return sfail(MS_ERR_INVALID_ARG, "out or a 256-byte aligned workspace missing");
    smd_plan *p = new (std::nothrow) smd_plan;
    if (!p) return sfail(MS_ERR_INVALID_ARG, "out of host memory");
    p->n = pb->n;
    p->n2 = pb->n * pb->n;
    p->M = pb->n_slices;
    p->S = pb->n_pos;
    p->dx = pb->pixel_size;
    p->lambda = pb->wavelength;
    p->dz.assign(pb->dz ? pb->dz : nullptr, pb->dz ? pb->dz + std::max(p->M - 1, 0) : nullptr);
    for (long long i = 0; i < p->S; ++i) {
        p->pos.push_back((int)pb->positions[2 * i]);
        p->pos.push_back((int)pb->positions[2 * i + 1]);
    }
    plan_layout(*p);
    if (ws_bytes < p->total) {
        const size_t need = p->total;
        delete p;
        return sfail(MS_ERR_BUDGET, "workspace too small: " + std::to_string(need) + " bytes needed");
    }
    p->ws = static_cast<char *>(workspace);
    if (rocblas_create_handle(&p->h) != rocblas_status_success) {
        delete p;
        return sfail(MS_ERR_HIP, "rocblas_create_handle failed");
    }
    rocblas_set_workspace(p->h, p->at<char>(p->blas), kBlasWorkspace);
    *out = p;
    return MS_OK;
}

void smd_plan_destroy(smd_plan *p)
{
    if (!p) return;
    if (p->h) rocblas_destroy_handle(p->h);
    delete p;
}

int32_t smd_set_probe(smd_plan *p, hipStream_t st, const void *probe)
{
    if (!p || !probe) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    rocblas_set_stream(p->h, st);
    const long long n2 = p->n2, S = p->S;
    const int n = p->n;
    float2 *F = p->at<float2>(p->F);
    dft_kernel<<<blocks(n2 * n2), 256, 0, st>>>(F, n);
    for (int m = 0; m + 1 < p->M; ++m) {
        h_rows_kernel<<<blocks(n2 * n2), 256, 0, st>>>(F, p->at<float2>(p->T1), n, p->dz[m], p->lambda, p->dx);
        // G = F^H (diag(h) F) / N^2
        if (!gemm(p, H_, N_, p->n2, p->n2, p->n2, std::complex<float>(1.0f / (float)n2, 0.f), F, p->n2,
                  p->at<float2>(p->T1), p->n2, 0.0f, p->at<float2>(p->G) + (size_t)m * p->mat(), p->n2))
            return MS_ERR_HIP;
    }
    if (hipMemcpyAsync(p->at<int2>(p->posd), p->pos.data(), (size_t)S * 8, hipMemcpyHostToDevice, st) != hipSuccess)
        return sfail(MS_ERR_HIP, "position upload failed");
    float2 *P = p->at<float2>(p->P);
    probe_matrix_kernel<<<blocks(n2 * S), 256, 0, st>>>(static_cast<const float2 *>(probe), p->at<int2>(p->posd), P,
                                                          n, S);
    // Gram matrix P^H P (S x S) into Z (n2 x S >= S x S when S <= n2, else into X / U region)
    const bool fits = S * S <= (long long)p->mat();
    float2 *gram = fits ? p->at<float2>(p->X) : nullptr;
    if (!gram) return sfail(MS_ERR_UNSUPPORTED, "more positions than N^2 x N^2 / S entries");
    if (!gemm(p, H_, N_, (int)S, (int)S, p->n2, 1.0f, P, (int)S, P, (int)S, 0.0f, gram, (int)S))
        return MS_ERR_HIP;
    std::vector<std::complex<float>> g((size_t)S * S);
    if (hipMemcpyAsync(g.data(), gram, g.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return sfail(MS_ERR_HIP, "Gram matrix download failed");
    // largest eigenvalue of the Hermitian PSD Gram matrix: power iteration with Rayleigh quotients
    std::vector<std::complex<double>> v((size_t)S, std::complex<double>(1.0, 0.0)), w((size_t)S);
    double ev = 0.0;
    for (int it = 0; it < 5000; ++it) {
        double nrm = 0.0;
        for (long long i = 0; i < S; ++i) nrm += std::norm(v[i]);
        nrm = std::sqrt(nrm);
        for (auto &x : v) x /= nrm;
        for (long long i = 0; i < S; ++i) {
            std::complex<double> acc = 0.0;
            for (long long j = 0; j < S; ++j) acc += std::complex<double>(g[(size_t)i * S + j]) * v[j];
            w[i] = acc;
        }
        double rq = 0.0;
        for (long long i = 0; i < S; ++i) rq += (std::conj(v[i]) * w[i]).real();
        // the Rayleigh quotient's error is quadratic in the eigenvector's: 1e-12 is far below FP32
        const bool done = it > 10 && std::fabs(rq - ev) <= 1e-12 * rq;
        ev = rq;
        v.swap(w);
        if (done) break;
    }
    p->mu_a = ev > 0.0 ? 1.0 / ((double)n2 * ev) : 0.0;
    p->ready = true;
    return hip_ok("smd_set_probe");
}

int32_t smd_compose(smd_plan *p, hipStream_t st, const void *slices, const double *lambda, void *a_out)
{
    if (!p || !slices || !lambda || !a_out) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    if (!p->ready) return sfail(MS_ERR_INVALID_ARG, "call smd_set_probe first");
    rocblas_set_stream(p->h, st);
    if (!compose_into(p, st, static_cast<const float2 *>(slices),
                      std::complex<float>((float)lambda[0], (float)lambda[1]), static_cast<float2 *>(a_out)))
        return MS_ERR_HIP;
    return hip_ok("smd_compose");
}

int32_t smd_estimate(smd_plan *p, hipStream_t st, const float *measured, void *a, int32_t steps, double *loss_first)
{
    if (!p || !measured || !a) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    if (!p->ready) return sfail(MS_ERR_INVALID_ARG, "call smd_set_probe first");
    if (steps < 0) return sfail(MS_ERR_INVALID_ARG, "steps must be >= 0");
    rocblas_set_stream(p->h, st);
    const int n2 = p->n2, S = (int)p->S;
    float2 *A = static_cast<float2 *>(a), *F = p->at<float2>(p->F), *P = p->at<float2>(p->P);
    float2 *Z = p->at<float2>(p->Z), *R = p->at<float2>(p->R);
    double *part = p->at<double>(p->part);
    for (int k = 0; k < steps; ++k) {
        // F (A P): the product with the N^2 x S probe matrix first, 2 N^4 S instead of N^6 + N^4 S
        if (!gemm(p, N_, N_, n2, S, n2, 1.0f, A, n2, P, S, 0.0f, R, S)) return MS_ERR_HIP;          // A P
        if (!gemm(p, N_, N_, n2, S, n2, 1.0f, F, n2, R, S, 0.0f, Z, S)) return MS_ERR_HIP;          // F A P
        smd_residual_kernel<<<kRed, 256, 0, st>>>(Z, measured, n2, S, part);
        if (k == 0 && loss_first) half_sum_kernel<<<1, 1, 0, st>>>(part, kRed, loss_first);
        if (!gemm(p, H_, N_, n2, S, n2, 1.0f, F, n2, Z, S, 0.0f, R, S)) return MS_ERR_HIP;          // F^H r
        if (!gemm(p, N_, H_, n2, n2, S, std::complex<float>((float)-p->mu_a, 0.f), R, S, P, S, 1.0f, A, n2))
            return MS_ERR_HIP;                                                                     // A -= mu (F^H r) P^H
    }
    return hip_ok("smd_estimate");
}

int32_t smd_decompose(smd_plan *p, hipStream_t st, const void *a_hat, void *slices, double *lambda, void *a_tilde_out)
{
    if (!p || !a_hat || !slices || !lambda) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    if (!p->ready) return sfail(MS_ERR_INVALID_ARG, "call smd_set_probe first");
    rocblas_set_stream(p->h, st);
    const int n2 = p->n2, M = p->M;
    const long long nn = (long long)n2 * n2;
    const float2 *Ah = static_cast<const float2 *>(a_hat);
    float2 *sl = static_cast<float2 *>(slices);
    float2 *old = p->at<float2>(p->old);
    const std::complex<float> lam((float)lambda[0], (float)lambda[1]);
    if (hipMemcpyAsync(old, sl, (size_t)M * n2 * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return sfail(MS_ERR_HIP, "slice copy failed");
    peak_kernel<<<M, 256, 0, st>>>(old, n2, p->at<double>(p->peak));
    const float2 one = make_float2(1.f, 0.f);
    float2 *pfx = p->at<float2>(p->pfx), *sfx = p->at<float2>(p->sfx);
    auto G = [&](int m) { return p->at<float2>(p->G) + (size_t)m * p->mat(); };
    // suffixes S_0 = I, S_{l+1} = G_l O_l S_l; prefixes R_{M-1} = I, R_l = R_{l+1} O_{l+1} G_l
    set_diag_kernel<<<blocks(nn), 256, 0, st>>>(sfx, nullptr, n2, one);
    for (int l = 0; l + 1 < M; ++l) {
        diag_scale_kernel<<<blocks(nn), 256, 0, st>>>(p->at<float2>(p->T1), sfx + (size_t)l * nn, old + (size_t)l * n2,
                                                      n2, 1, one);
        if (!gemm(p, N_, N_, n2, n2, n2, 1.0f, G(l), n2, p->at<float2>(p->T1), n2, 0.0f, sfx + (size_t)(l + 1) * nn, n2))
            return MS_ERR_HIP;
    }
    set_diag_kernel<<<blocks(nn), 256, 0, st>>>(pfx + (size_t)(M - 1) * nn, nullptr, n2, one);
    for (int l = M - 2; l >= 0; --l) {
        diag_scale_kernel<<<blocks(nn), 256, 0, st>>>(p->at<float2>(p->T1), pfx + (size_t)(l + 1) * nn,
                                                      old + (size_t)(l + 1) * n2, n2, 0, one);
        if (!gemm(p, N_, N_, n2, n2, n2, 1.0f, p->at<float2>(p->T1), n2, G(l), n2, 0.0f, pfx + (size_t)l * nn, n2))
            return MS_ERR_HIP;
    }
    float2 *X = p->at<float2>(p->X), *U = p->at<float2>(p->U), *Y = p->at<float2>(p->T2);
    double2 *grad = p->at<double2>(p->grad);
    for (int l = 0; l < M; ++l) {
        float2 *Rl = pfx + (size_t)l * nn, *Sl = sfx + (size_t)l * nn;
        diag_scale_kernel<<<blocks(nn), 256, 0, st>>>(Y, Rl, old + (size_t)l * n2, n2, 0, one);   // R_l O_l
        if (hipMemcpyAsync(X, Ah, (size_t)nn * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return sfail(MS_ERR_HIP, "copy failed");
        if (!gemm(p, N_, N_, n2, n2, n2, lam, Y, n2, Sl, n2, -1.0f, X, n2)) return MS_ERR_HIP;   // lambda R O S - A_hat
        if (!gemm(p, H_, N_, n2, n2, n2, 1.0f, Rl, n2, X, n2, 0.0f, U, n2)) return MS_ERR_HIP;   // R^H X
        row_dot_conj_kernel<<<n2, 256, 0, st>>>(U, Sl, n2, grad);                               // diag(R^H X S^H)
        prox_update_kernel<<<1, 256, 0, st>>>(old + (size_t)l * n2, grad, p->at<double>(p->peak), M, l, lambda[0],
                                              lambda[1], n2, sl + (size_t)l * n2);
    }
    float2 *At = a_tilde_out ? static_cast<float2 *>(a_tilde_out) : X;
    if (!compose_into(p, st, sl, 1.0f, At)) return MS_ERR_HIP;
    double *part = p->at<double>(p->part);
    trace_kernel<<<kRed, 256, 0, st>>>(At, Ah, nn, part);
    std::vector<double> h((size_t)kRed * 3);
    if (hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return sfail(MS_ERR_HIP, "trace download failed");
    double tr = 0.0, ti = 0.0, tt = 0.0;
    for (int i = 0; i < kRed; ++i) {
        tr += h[3 * i];
        ti += h[3 * i + 1];
        tt += h[3 * i + 2];
    }
    if (tt > 0.0) {
        lambda[0] = tr / tt;
        lambda[1] = ti / tt;
    }
    return hip_ok("smd_decompose");
}

int32_t smd_result(smd_plan *p, hipStream_t st, const void *slices, const double *lambda, void *out)
{
    if (!p || !slices || !lambda || !out) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    const std::complex<double> root = std::pow(std::complex<double>(lambda[0], lambda[1]), 1.0 / p->M);
    const long long count = (long long)p->M * p->n2;
    scale_kernel<<<blocks(count), 256, 0, st>>>(static_cast<float2 *>(out), static_cast<const float2 *>(slices), count,
                                                root.real(), root.imag());
    return hip_ok("smd_result");
}

const char *smd_last_error(void) { return s_err.c_str(); }

}  // extern "C"
