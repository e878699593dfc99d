// Host runtime and C ABI of the gfx950 pooled-pCN tomography library.
//
// Owns every device buffer behind a qst_problem handle, validates arguments,
// picks a launch shape per qubit count, and turns each call of the ABI into
// kernel launches on the caller's stream.  See include/qst.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qst.h"
#include "acf_kernel.hpp"
#include "batch_kernel.hpp"
#include "chain_kernel.hpp"
#include "da_kernel.hpp"
#include "mlp_kernels.hpp"
#include "pool_kernel.hpp"

namespace {

thread_local std::string g_err;

struct QstError {
    qst_status code;
    std::string msg;
};

[[noreturn]] void fail(qst_status code, const std::string& msg) { throw QstError{code, msg}; }

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) fail(QST_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// A caller-owned device buffer: device memory of `device` with at least
// `bytes` bytes from p to the end of its allocation (an allocator may hand
// out part of a larger allocation, so a buffer that is too small but lies
// inside a larger block passes; host memory, another device's memory and
// overruns past the allocation are refused).
void check_device_buffer(const void* p, size_t bytes, int device, const char* what)
{
    if (bytes == 0) return;
    if (!p) fail(QST_ERR_INVALID, std::string(what) + " is NULL");
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        fail(QST_ERR_INVALID, std::string(what) + " is not device memory");
    }
    if (at.type != hipMemoryTypeDevice) fail(QST_ERR_INVALID, std::string(what) + " is not device memory");
    if (at.device != device) fail(QST_ERR_INVALID, std::string(what) + " is on another device");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
        (void)hipGetLastError();
        fail(QST_ERR_INVALID, std::string(what) + ": allocation not found");
    }
    const size_t off = static_cast<size_t>(static_cast<const char*>(p) - static_cast<const char*>(base));
    if (off > size || bytes > size - off)
        fail(QST_ERR_INVALID, std::string(what) + " is smaller than the call needs");
}

int current_device()
{
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    return dev;
}

// Dynamic LDS above the default limit must be allowed per kernel and per
// device once; a larger request later raises the allowance.
void allow_dynamic_lds(const void* kernel, size_t bytes)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> allowed;
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lock(mu);
    size_t& cur = allowed[{kernel, dev}];
    if (cur >= bytes) return;
    hip_check(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)),
              "hipFuncSetAttribute");
    cur = bytes;
}

template <typename F>
qst_status guarded(F&& f)
{
    try {
        f();
        g_err.clear();
        return QST_OK;
    } catch (const QstError& e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return QST_ERR_NOMEM;
    } catch (...) {
        g_err = "unexpected internal error";
        return QST_ERR_DEVICE;
    }
}

template <typename T>
T* dev_alloc(size_t n)
{
    if (n == 0) n = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(QST_ERR_NOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return static_cast<T*>(p);
}

template <typename T>
void dev_free(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

int ipow3(int q)
{
    int k = 1;
    for (int i = 0; i < q; ++i) k *= 3;
    return k;
}

// ---------------------------------------------------------------------------
// The Pauli measurement matrix of the dense path, built exactly on the host.
// Row kl = k D + l holds Tr(Lambda_kl rho) as a linear form of packed rho:
// p = sum_a rho_aa Pi_aa + sum_{a<b} 2 (Re rho_ab Re Pi_ab + Im rho_ab Im Pi_ab)
// with Pi = Lambda_kl = (x)_q pi_{s_q b_q}.  Every entry is 0 or +-2^-j, exact in
// FP64, FP32 and BF16.
// ---------------------------------------------------------------------------
std::complex<double> qubit_projector(int s, int b, int x, int y)
{
    if (s == 2) return (x == b && y == b) ? 1.0 : 0.0;          // Z: |b><b|
    const double sgn = b == 0 ? 1.0 : -1.0;                     // b = 0: eigenvalue +1
    if (x == y) return 0.5;
    if (s == 0) return 0.5 * sgn;                               // X: (1/2)[[1, +-1], [+-1, 1]]
    return x == 0 ? std::complex<double>(0.0, -0.5 * sgn)       // Y: (1/2)[[1, -+i], [+-i, 1]]
                  : std::complex<double>(0.0, 0.5 * sgn);
}

std::vector<double> pauli_matrix_packed(int Q)
{
    const int D = 1 << Q, D2 = D * D, K = ipow3(Q);
    std::vector<double> M(static_cast<size_t>(K) * D * D2);
    std::vector<int> s(Q), bq(Q);
    for (int k = 0; k < K; ++k) {
        for (int q = Q - 1, kk = k; q >= 0; --q) { s[q] = kk % 3; kk /= 3; }
        for (int l = 0; l < D; ++l) {
            for (int q = 0; q < Q; ++q) bq[q] = (l >> (Q - 1 - q)) & 1;
            auto Pi = [&](int a, int b) {
                std::complex<double> v = 1.0;
                for (int q = 0; q < Q; ++q) v *= qubit_projector(s[q], bq[q], (a >> (Q - 1 - q)) & 1, (b >> (Q - 1 - q)) & 1);
                return v;
            };
            double* row = M.data() + static_cast<size_t>(k * D + l) * D2;
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c)
                    row[r * D + c] = r == c ? Pi(r, r).real() : (r < c ? 2.0 * Pi(r, c).real() : 2.0 * Pi(c, r).imag());
        }
    }
    return M;
}

// M in MFMA A-operand fragment order (see the dense contraction in
// chain_kernel.hpp), as raw bytes of the requested precision.
// The packed-real measurement matrix of user POVM elements (n complex D x D
// matrices, row-major, interleaved), padded with zero rows to 3^Q 2^Q:
// p_m = Tr(Pi_m rho) = sum_a Re Pi_aa rho_aa + sum_{a<b} 2 (Re Pi_ab Re rho_ab +
// Im Pi_ab Im rho_ab), so row m holds Re Pi_aa at (a, a), 2 Re Pi_ab at (a, b)
// and 2 Im Pi_ab at (b, a) for a < b, against the packed form of rho.
std::vector<double> povm_matrix_packed(int Q, const double* povm, int n)
{
    const int D = 1 << Q, D2 = D * D, KD = ipow3(Q) * D;
    std::vector<double> M(static_cast<size_t>(KD) * D2, 0.0);
    for (int m = 0; m < n; ++m) {
        const double* P = povm + static_cast<size_t>(m) * 2 * D2;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                const double re = P[2 * (a * D + b)], im = P[2 * (a * D + b) + 1];
                const double re_t = P[2 * (b * D + a)], im_t = P[2 * (b * D + a) + 1];
                if (!std::isfinite(re) || !std::isfinite(im)) fail(QST_ERR_INVALID, "POVM element not finite");
                if (std::fabs(re - re_t) > 1e-12 || std::fabs(im + im_t) > 1e-12)
                    fail(QST_ERR_INVALID, "POVM element not Hermitian");
                double* row = M.data() + static_cast<size_t>(m) * D2;
                if (a == b) row[a * D + a] = re;
                else if (a < b) {
                    row[a * D + b] = 2.0 * re;
                    row[b * D + a] = 2.0 * im;
                }
            }
    }
    return M;
}

// Packed weights of Lambda = sum_m lambda_m Pi_m for the linear part of the
// Poisson log-likelihood (sum_m lambda_m p_m = Tr(rho Lambda)): W[a][a] =
// Lambda_aa, W[a][b] = 2 Re Lambda_ab and W[b][a] = 2 Im Lambda_ab for a < b,
// so that Tr(rho Lambda) = sum_k W[k] (packed rho)[k].  Pauli settings:
// Lambda accumulated from the product eigenvectors e_kl (Pi_kl = e e^dag);
// user POVM elements: the rows of their packed matrix M weighted by lambda.
std::vector<double> linear_weights_packed(int Q, const double* lambda, int n, const std::vector<double>& povm_M)
{
    const int D = 1 << Q, D2 = D * D, K = ipow3(Q);
    std::vector<double> W(D2, 0.0);
    if (!povm_M.empty()) {
        for (int m = 0; m < n; ++m)
            for (int k = 0; k < D2; ++k) W[k] += lambda[m] * povm_M[static_cast<size_t>(m) * D2 + k];
        return W;
    }
    // one qubit's eigenvectors: X (1, +-1)/sqrt 2, Y (1, +-i)/sqrt 2, Z e_0 / e_1
    auto comp = [](int s, int b, int x) -> std::complex<double> {
        const double r = 0.70710678118654752440;
        const double sgn = b == 0 ? 1.0 : -1.0;
        if (s == 2) return x == b ? 1.0 : 0.0;
        if (x == 0) return r;
        return s == 0 ? std::complex<double>(sgn * r, 0.0) : std::complex<double>(0.0, sgn * r);
    };
    std::vector<std::complex<double>> L(static_cast<size_t>(D2), 0.0), e(D);
    for (int k = 0; k < K; ++k) {
        int dig[8];
        for (int q = Q - 1, kk = k; q >= 0; --q) { dig[q] = kk % 3; kk /= 3; }
        for (int l = 0; l < D; ++l) {
            const double lam = lambda[k * D + l];
            if (lam == 0.0) continue;
            for (int a = 0; a < D; ++a) {
                std::complex<double> v = 1.0;
                for (int q = 0; q < Q; ++q) v *= comp(dig[q], (l >> (Q - 1 - q)) & 1, (a >> (Q - 1 - q)) & 1);
                e[a] = v;
            }
            for (int a = 0; a < D; ++a)
                for (int b = a; b < D; ++b) L[static_cast<size_t>(a) * D + b] += lam * e[a] * std::conj(e[b]);
        }
    }
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) {
            const std::complex<double> v = L[static_cast<size_t>(a) * D + b];
            if (a == b) W[a * D + a] = v.real();
            else {
                W[a * D + b] = 2.0 * v.real();
                W[b * D + a] = 2.0 * v.imag();
            }
        }
    return W;
}

// The measurement matrix in the dense kernels' MFMA operand order.
std::vector<uint8_t> matrix_fragments(int Q, const std::vector<double>& M, int prec)
{
    const int D = 1 << Q, D2 = D * D, KD = ipow3(Q) * D;
    const int NT = (KD + 15) / 16;
    auto m_at = [&](int row, int col) { return (row < KD && col < D2) ? M[static_cast<size_t>(row) * D2 + col] : 0.0; };
    std::vector<uint8_t> out;
    if (prec == qst::kPrecF64 || prec == qst::kPrecF32) {
        const int KS = D2 / 4;
        const size_t n = static_cast<size_t>(NT) * KS * 64;
        out.resize(n * (prec == qst::kPrecF64 ? 8 : 4));
        for (int nt = 0; nt < NT; ++nt)
            for (int ks = 0; ks < KS; ++ks)
                for (int l = 0; l < 64; ++l) {
                    const double v = m_at(16 * nt + l % 16, 4 * ks + l / 16);
                    const size_t i = (static_cast<size_t>(nt) * KS + ks) * 64 + l;
                    if (prec == qst::kPrecF64) reinterpret_cast<double*>(out.data())[i] = v;
                    else reinterpret_cast<float*>(out.data())[i] = static_cast<float>(v);
                }
    } else {
        const int KS = (D2 + 31) / 32;
        const size_t n = static_cast<size_t>(NT) * KS * 64 * 8;
        out.resize(n * 2);
        uint16_t* h = reinterpret_cast<uint16_t*>(out.data());
        for (int nt = 0; nt < NT; ++nt)
            for (int ks = 0; ks < KS; ++ks)
                for (int l = 0; l < 64; ++l)
                    for (int v = 0; v < 8; ++v) {
                        const float f = static_cast<float>(m_at(16 * nt + l % 16, 32 * ks + 8 * (l / 16) + v));
                        uint32_t bits;
                        std::memcpy(&bits, &f, 4);
                        if ((bits & 0xFFFFu) != 0) fail(QST_ERR_DEVICE, "measurement matrix entry not exact in BF16");
                        h[((static_cast<size_t>(nt) * KS + ks) * 64 + l) * 8 + v] = static_cast<uint16_t>(bits >> 16);
                    }
    }
    return out;
}

// Launch shape of the chain kernel for one qubit count: team size G (threads
// per chain) and workgroup size WG.
struct Shape {
    int G, WG;
};

// Shapes with a compiled single-problem chain kernel (Kronecker path).
constexpr Shape kShapes[7][5] = {
    {},
    {{8, 64}, {16, 64}, {64, 64}},
    {{16, 64}, {32, 64}, {64, 64}},
    {{32, 64}, {64, 64}},
    {{64, 64}, {64, 256}},
    {{64, 64}, {128, 128}, {256, 256}, {512, 512}},
    {{256, 256}, {512, 512}, {1024, 1024}},
};

// Current choice per qubit count (set by qst_set_launch_shape, e.g. from the
// autotuner's table).
Shape g_shape[7] = {{0, 0}, {8, 64}, {16, 64}, {32, 64}, {64, 256}, {256, 256}, {1024, 1024}};

Shape current_shape(int Q) { return g_shape[Q]; }

// Path that QST_PATH_AUTO takes per qubit count and precision: the Kronecker
// route, except BF16x3 (dense only); the autotuner installs its measured
// choice through qst_set_auto_path.
qst_path g_auto_path[7][3] = {
    {QST_PATH_KRON, QST_PATH_KRON, QST_PATH_DENSE}, {QST_PATH_KRON, QST_PATH_KRON, QST_PATH_DENSE},
    {QST_PATH_KRON, QST_PATH_KRON, QST_PATH_DENSE}, {QST_PATH_KRON, QST_PATH_KRON, QST_PATH_DENSE},
    {QST_PATH_KRON, QST_PATH_KRON, QST_PATH_DENSE}, {QST_PATH_KRON, QST_PATH_KRON, QST_PATH_DENSE},
    {QST_PATH_KRON, QST_PATH_KRON, QST_PATH_DENSE}};

bool shape_compiled(int Q, Shape sh)
{
    for (const Shape& c : kShapes[Q])
        if (c.G == sh.G && c.WG == sh.WG && c.G > 0) return true;
    return false;
}

// a.R is one past the last problem-wide chain index, chain0 the first (make_args)
// restore: the kernel that evaluates restored states instead of the steps
template <int Q, int G, int WG, int PATH, int PREC, int PARAM = qst::kParamGamma>
void launch_chains_t(const qst::ChainArgs& a, int64_t chain0, hipStream_t s, bool restore)
{
    using S = qst::TeamShape<Q, G, PATH, PARAM>;
    const int64_t teams = WG / G;
    const int64_t blocks = (a.R - chain0 + teams - 1) / teams;
    const size_t lds = (static_cast<size_t>(teams) * S::kLdsChain + qst::WgTables<Q, PATH>::kDoubles) * sizeof(double);
    if (blocks > 0x7fffffff) fail(QST_ERR_INVALID, "too many chains for one launch");
    if (restore) {
        allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_chains_restore<Q, G, WG, PATH, PREC, PARAM>), lds);
        hipLaunchKernelGGL((qst::k_chains_restore<Q, G, WG, PATH, PREC, PARAM>), dim3(static_cast<unsigned>(blocks)),
                           dim3(WG), lds, s, a, chain0);
    } else {
        allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_chains<Q, G, WG, PATH, PREC, PARAM>), lds);
        hipLaunchKernelGGL((qst::k_chains<Q, G, WG, PATH, PREC, PARAM>), dim3(static_cast<unsigned>(blocks)),
                           dim3(WG), lds, s, a, chain0);
    }
    hip_check(hipGetLastError(), "chain kernel launch");
}

template <int Q, int PREC>
void launch_loglik_dense_t(const double* nd, const void* mfrag, const double* rho, int64_t n, double* out,
                           int poisson, hipStream_t s)
{
    using SH = qst::DenseAloneShape<Q, PREC>;
    const int64_t blocks = (n + SH::kStates - 1) / SH::kStates;
    if (blocks > 0x7fffffff) fail(QST_ERR_INVALID, "too many matrices for one launch");
    const size_t lds = SH::kLdsBytes;
    allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_loglik_dense<Q, PREC>), lds);
    hipLaunchKernelGGL((qst::k_loglik_dense<Q, PREC>), dim3(static_cast<unsigned>(blocks)), dim3(1024), lds, s, nd,
                       mfrag, rho, n, out, poisson);
    hip_check(hipGetLastError(), "dense loglik kernel launch");
}

template <int Q, int G, int WG, int PREC>
void launch_loglik_t(const double* nd, const uint16_t* mu, const double* ndv, const uint16_t* muv, const double* rho,
                     int64_t n, double* out, int poisson, hipStream_t s)
{
    using S = qst::TeamShape<Q, G>;
    const int64_t teams = WG / G;
    const int64_t blocks = (n + teams - 1) / teams;
    const size_t lds = (static_cast<size_t>(teams) * S::kLds + qst::WgTables<Q>::kDoubles) * sizeof(double);
    allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_loglik<Q, G, WG, PREC>), lds);
    if (blocks > 0x7fffffff) fail(QST_ERR_INVALID, "too many states for one launch");
    hipLaunchKernelGGL((qst::k_loglik<Q, G, WG, PREC>), dim3(static_cast<unsigned>(blocks)), dim3(WG), lds, s, nd,
                       mu, ndv, muv, rho, n, out, poisson);
    hip_check(hipGetLastError(), "loglik kernel launch");
}

// Dirichlet(alpha) weights: the Kronecker route with the default team shape
// of each qubit count.
void launch_chains_dirichlet(int Q, int prec, const qst::ChainArgs& a, int64_t chain0, hipStream_t s,
                             bool restore = false)
{
    using namespace qst;
#define QST_DIR(q, g, wg)                                                                               \
    if (Q == q)                                                                                         \
        return prec == kPrecF32 ? launch_chains_t<q, g, wg, kPathKron, kPrecF32, kParamDirichlet>(a, chain0, s, restore) \
                                : launch_chains_t<q, g, wg, kPathKron, kPrecF64, kParamDirichlet>(a, chain0, s, restore);
    QST_DIR(1, 8, 64) QST_DIR(2, 16, 64) QST_DIR(3, 32, 64) QST_DIR(4, 64, 256) QST_DIR(5, 256, 256)
    QST_DIR(6, 1024, 1024)
#undef QST_DIR
    fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
}

// Algorithm 1 (the Bures draw): the Kronecker route with one fixed team
// shape per qubit count (one wavefront per chain at 4 qubits).
void launch_chains_bures(int Q, int prec, const qst::ChainArgs& a, int64_t chain0, hipStream_t s,
                         bool restore = false)
{
    using namespace qst;
#define QST_BURES(q, g, wg)                                                                             \
    if (Q == q)                                                                                         \
        return prec == kPrecF32 ? launch_chains_t<q, g, wg, kPathKron, kPrecF32, kParamBures>(a, chain0, s, restore)     \
                                : launch_chains_t<q, g, wg, kPathKron, kPrecF64, kParamBures>(a, chain0, s, restore);
    QST_BURES(1, 8, 64) QST_BURES(2, 16, 64) QST_BURES(3, 32, 64) QST_BURES(4, 64, 256)
#undef QST_BURES
    fail(QST_ERR_UNSUPPORTED, "Algorithm 1 (QST_PARAM_BURES) is built for 1..4 qubits");
}

void launch_chains(int Q, Shape sh, int path, int prec, const qst::ChainArgs& a, int64_t chain0, hipStream_t s,
                   bool restore = false)
{
    using namespace qst;
    if (path == kPathDense) {
#define QST_DENSE(q, pr) \
    if (Q == q && prec == pr) return launch_chains_t<q, 64, 1024, kPathDense, pr>(a, chain0, s, restore);
        QST_DENSE(1, kPrecF64) QST_DENSE(1, kPrecF32) QST_DENSE(1, kPrecBF16x3)
        QST_DENSE(2, kPrecF64) QST_DENSE(2, kPrecF32) QST_DENSE(2, kPrecBF16x3)
        QST_DENSE(3, kPrecF64) QST_DENSE(3, kPrecF32) QST_DENSE(3, kPrecBF16x3)
        QST_DENSE(4, kPrecF64) QST_DENSE(4, kPrecF32) QST_DENSE(4, kPrecBF16x3)
#undef QST_DENSE
        fail(QST_ERR_UNSUPPORTED, "dense contraction is built for 1..4 qubits only");
    }
#define QST_CASE(q, g, wg)                                                                              \
    if (Q == q && sh.G == g && sh.WG == wg)                                                             \
        return prec == kPrecF32 ? launch_chains_t<q, g, wg, kPathKron, kPrecF32>(a, chain0, s, restore)         \
                                : launch_chains_t<q, g, wg, kPathKron, kPrecF64>(a, chain0, s, restore);
    QST_CASE(1, 8, 64) QST_CASE(1, 16, 64) QST_CASE(1, 64, 64)
    QST_CASE(2, 16, 64) QST_CASE(2, 32, 64) QST_CASE(2, 64, 64)
    QST_CASE(3, 32, 64) QST_CASE(3, 64, 64)
    QST_CASE(4, 64, 64) QST_CASE(4, 64, 256)
    QST_CASE(5, 64, 64) QST_CASE(5, 128, 128) QST_CASE(5, 256, 256) QST_CASE(5, 512, 512)
    QST_CASE(6, 256, 256) QST_CASE(6, 512, 512) QST_CASE(6, 1024, 1024)
#undef QST_CASE
    fail(QST_ERR_UNSUPPORTED, "no chain kernel for Q=" + std::to_string(Q) + " G=" + std::to_string(sh.G));
}

void launch_loglik_dense(int Q, int prec, const double* nd, const void* mfrag, const double* rho, int64_t n,
                         double* out, int poisson, hipStream_t s)
{
    using namespace qst;
#define QST_DENSE(q, pr) \
    if (Q == q && prec == pr) return launch_loglik_dense_t<q, pr>(nd, mfrag, rho, n, out, poisson, s);
    QST_DENSE(1, kPrecF64) QST_DENSE(1, kPrecF32) QST_DENSE(1, kPrecBF16x3)
    QST_DENSE(2, kPrecF64) QST_DENSE(2, kPrecF32) QST_DENSE(2, kPrecBF16x3)
    QST_DENSE(3, kPrecF64) QST_DENSE(3, kPrecF32) QST_DENSE(3, kPrecBF16x3)
    QST_DENSE(4, kPrecF64) QST_DENSE(4, kPrecF32) QST_DENSE(4, kPrecBF16x3)
    QST_DENSE(5, kPrecF64) QST_DENSE(5, kPrecF32) QST_DENSE(5, kPrecBF16x3)
#undef QST_DENSE
    fail(QST_ERR_UNSUPPORTED, "the dense contraction is built for 1..5 qubits");
}

template <int PREC>
void launch_loglik_p(int Q, const double* nd, const uint16_t* mu, const double* ndv, const uint16_t* muv,
                     const double* rho, int64_t n, double* out, int poisson, hipStream_t s)
{
    switch (Q) {
        case 1: return launch_loglik_t<1, 8, 64, PREC>(nd, mu, ndv, muv, rho, n, out, poisson, s);
        case 2: return launch_loglik_t<2, 16, 64, PREC>(nd, mu, ndv, muv, rho, n, out, poisson, s);
        case 3: return launch_loglik_t<3, 32, 64, PREC>(nd, mu, ndv, muv, rho, n, out, poisson, s);
        case 4: return launch_loglik_t<4, 64, 64, PREC>(nd, mu, ndv, muv, rho, n, out, poisson, s);
        case 5: return launch_loglik_t<5, 64, 64, PREC>(nd, mu, ndv, muv, rho, n, out, poisson, s);
        case 6: return launch_loglik_t<6, 256, 256, PREC>(nd, mu, ndv, muv, rho, n, out, poisson, s);
    }
    fail(QST_ERR_INVALID, "bad Q");
}

void launch_loglik(int Q, int prec, const double* nd, const uint16_t* mu, const double* ndv, const uint16_t* muv,
                   const double* rho, int64_t n, double* out, int poisson, hipStream_t s)
{
    if (prec == qst::kPrecF32) return launch_loglik_p<qst::kPrecF32>(Q, nd, mu, ndv, muv, rho, n, out, poisson, s);
    return launch_loglik_p<qst::kPrecF64>(Q, nd, mu, ndv, muv, rho, n, out, poisson, s);
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free pooling call (qst_pool_moments_static):
// one file-scope array per device for the partial sums of the fixed-order
// reduction.  In host code `scratch` only names the symbol; its device
// address, per device, comes from hipGetSymbolAddress at set-up (the first
// qst_init_problem on that device) and is the only way host code refers to it.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// With `dev` current: look up (once) and return its copy of `scratch`.
void* scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) fail(QST_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) fail(QST_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

struct DeviceGuard {
    int prev = 0;
    explicit DeviceGuard(int dev)
    {
        hip_check(hipGetDevice(&prev), "hipGetDevice");
        hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceGuard() { (void)hipSetDevice(prev); }
};

}  // namespace

struct qst_problem {
    int Q = 0, D = 0, D2 = 0, d = 0, K = 0, KD = 0, device = 0;
    qst_precision precision = QST_FP64;
    qst_path path = QST_PATH_KRON;
    qst_param param = QST_PARAM_GAMMA;
    double alpha = 0.5;           // QST_PARAM_DIRICHLET: concentration of the weights
    std::vector<int64_t> counts;
    std::vector<double> povm_M;   // user POVM: packed measurement matrix (empty: the Pauli settings)
    bool poisson = false;  // Poisson counts with known intensities (else multinomial)
    double* nd = nullptr;  // counts as doubles [KD]; with Poisson counts followed by the packed weights W [D2]
    uint16_t* mu = nullptr;  // Pauli index of every (setting, transform position), [KD]
    double* ndv = nullptr;   // counts in the task-major order of the likelihood transforms, [KD]
    uint16_t* muv = nullptr; // Pauli indices in the same order, [KD]
    void* mfrag[3] = {nullptr, nullptr, nullptr};  // dense path: Pauli matrix fragments per precision

    const void* fragments(int prec)
    {
        if (!mfrag[prec]) {
            if (Q > 5) fail(QST_ERR_UNSUPPORTED, "the dense contraction is built for 1..5 qubits");
            const std::vector<uint8_t> f =
                matrix_fragments(Q, povm_M.empty() ? pauli_matrix_packed(Q) : povm_M, prec);
            void* d = dev_alloc<uint8_t>(f.size());
            hipError_t e = hipMemcpy(d, f.data(), f.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(d);
                fail(QST_ERR_DEVICE, std::string("copy Pauli matrix: ") + hipGetErrorString(e));
            }
            mfrag[prec] = d;
        }
        return mfrag[prec];
    }
    // chain state
    int64_t R = 0;
    int64_t chain0 = 0;     // index of chain 0 of this handle within its problem (qst_run_desc.chain_offset)
    bool reeval = false;    // qst_set_chain_state wrote x: evaluate log L and rho before the next run
    int64_t step = 0;
    bool have_run = false;
    double *x = nullptr, *ll = nullptr, *beta = nullptr, *rho = nullptr, *s1 = nullptr, *s2 = nullptr;
    int32_t* accw = nullptr;
    int64_t *nst = nullptr, *nacc = nullptr, *nnear = nullptr;
    hipStream_t last_stream = nullptr;
    // delayed acceptance (allocated on first use)
    int64_t da_R = 0;
    double *s_cur = nullptr, *yprop = nullptr, *u_mh = nullptr, *u_da = nullptr;
    int64_t* n_stage1 = nullptr;
    uint16_t* xb = nullptr;
    float* smlp = nullptr;
    int32_t *surv = nullptr, *n_surv = nullptr;

    int da_width() const { return (d + 31) / 32 * 32; }
    void free_da()
    {
        dev_free(s_cur);
        dev_free(yprop);
        dev_free(u_mh);
        dev_free(u_da);
        dev_free(n_stage1);
        dev_free(xb);
        dev_free(smlp);
        dev_free(surv);
        dev_free(n_surv);
        da_R = 0;
    }
    void ensure_da()
    {
        if (da_R == R) return;
        free_da();
        s_cur = dev_alloc<double>(R);
        yprop = dev_alloc<double>(static_cast<size_t>(R) * d);
        u_mh = dev_alloc<double>(R);
        u_da = dev_alloc<double>(R);
        n_stage1 = dev_alloc<int64_t>(R);
        xb = dev_alloc<uint16_t>(static_cast<size_t>(R) * da_width());
        smlp = dev_alloc<float>(R);
        surv = dev_alloc<int32_t>(R);
        n_surv = dev_alloc<int32_t>(1);
        da_R = R;
    }

    void free_state()
    {
        dev_free(x);
        dev_free(ll);
        dev_free(beta);
        dev_free(rho);
        dev_free(s1);
        dev_free(s2);
        dev_free(accw);
        dev_free(nst);
        dev_free(nacc);
        dev_free(nnear);
        free_da();
        R = 0;
    }
    void alloc_state(int64_t n)
    {
        free_state();
        x = dev_alloc<double>(static_cast<size_t>(n) * d);
        ll = dev_alloc<double>(n);
        beta = dev_alloc<double>(n);
        rho = dev_alloc<double>(static_cast<size_t>(n) * D2);
        s1 = dev_alloc<double>(static_cast<size_t>(n) * D2);
        s2 = dev_alloc<double>(static_cast<size_t>(n) * D2);
        accw = dev_alloc<int32_t>(n);
        nst = dev_alloc<int64_t>(n);
        nacc = dev_alloc<int64_t>(n);
        nnear = dev_alloc<int64_t>(n);
        R = n;
    }
};

namespace {

void validate_run(const qst_problem* p, const qst_run_desc& r)
{
    if (r.n_chains < 1) fail(QST_ERR_INVALID, "n_chains must be >= 1");
    if (r.n_steps < 0) fail(QST_ERR_INVALID, "n_steps must be >= 0");
    if (r.thin < 1) fail(QST_ERR_INVALID, "thin must be >= 1");
    if (r.burn_in < 0) fail(QST_ERR_INVALID, "burn_in must be >= 0");
    if (!(r.beta0 > 0.0 && r.beta0 <= 1.0)) fail(QST_ERR_INVALID, "beta0 must lie in (0, 1]");
    if (r.adapt_every < 0) fail(QST_ERR_INVALID, "adapt_every must be >= 0");
    if (r.adapt_every > 0 && !(r.adapt_factor > 0.0)) fail(QST_ERR_INVALID, "adapt_factor must be > 0");
    if (r.trace_chains < 0 || r.record_chains < 0 || r.record_every < 0)
        fail(QST_ERR_INVALID, "negative trace/record sizes");
    if (r.record_every > 0 && r.record_chains > 0 && !r.record_buf)
        fail(QST_ERR_INVALID, "record_buf is NULL");
    if (r.pair_every < 0 || r.pair_chains < 0) fail(QST_ERR_INVALID, "negative pair-recorder sizes");
    if (r.pair_every > 0 && r.pair_chains > 0 && (!r.pair_x || !r.pair_ll))
        fail(QST_ERR_INVALID, "pair buffers are NULL");
    if (r.pair_every > 0 && r.surrogate) fail(QST_ERR_UNSUPPORTED, "the pair recorder runs with plain pCN");
    if (r.surrogate && p->param != QST_PARAM_GAMMA)
        fail(QST_ERR_UNSUPPORTED, "delayed acceptance runs with the Gaussian/gamma parameterisation");
    if (r.surrogate && p->poisson)
        fail(QST_ERR_UNSUPPORTED, "delayed acceptance runs with the multinomial likelihood");
    // extents of what the kernels write into the caller's buffers
    const size_t steps = static_cast<size_t>(r.n_steps);
    const size_t tc = static_cast<size_t>(std::min<int64_t>(r.trace_chains, r.n_chains));
    if (r.trace_llprop) check_device_buffer(r.trace_llprop, tc * steps * sizeof(double), p->device, "trace_llprop");
    if (r.trace_logu) check_device_buffer(r.trace_logu, tc * steps * sizeof(double), p->device, "trace_logu");
    if (r.trace_accept) check_device_buffer(r.trace_accept, tc * steps, p->device, "trace_accept");
    if (r.record_every > 0 && r.record_chains > 0) {
        const size_t rc = static_cast<size_t>(std::min<int64_t>(r.record_chains, r.n_chains));
        check_device_buffer(r.record_buf, rc * (steps / r.record_every) * p->D2 * sizeof(double), p->device,
                            "record_buf");
    }
    if (r.pair_every > 0 && r.pair_chains > 0) {
        const size_t slots = steps / r.pair_every;
        const size_t pc = static_cast<size_t>(r.pair_chains);
        const size_t rows = slots > 0 ? (slots - 1) * pc + std::min<size_t>(pc, static_cast<size_t>(r.n_chains)) : 0;
        check_device_buffer(r.pair_x, rows * p->da_width() * sizeof(uint16_t), p->device, "pair_x");
        check_device_buffer(r.pair_ll, rows * sizeof(double), p->device, "pair_ll");
    }
    if (r.chain_offset < 0) fail(QST_ERR_INVALID, "chain_offset must be >= 0");
    if (r.chain_offset > 0 && r.chain_offset + r.n_chains + r.trace_chains + r.record_chains > 0x7fffffff)
        fail(QST_ERR_INVALID, "chain_offset + n_chains must stay below 2^31");
    if (r.chain_offset > 0 && r.pair_every > 0 && r.pair_chains > 0)
        fail(QST_ERR_UNSUPPORTED, "the pair recorder runs with chain_offset 0");
    if (r.resume) {
        if (!p->have_run) fail(QST_ERR_STATE, "resume requested before any run of this handle");
        if (r.n_chains != p->R) fail(QST_ERR_INVALID, "resume with a different n_chains");
        if (r.chain_offset != p->chain0) fail(QST_ERR_INVALID, "resume with a different chain_offset");
    }
    if (r.surrogate) {
        if (!r.surrogate->model) fail(QST_ERR_INVALID, "surrogate has no model (use qst_mlp_surrogate)");
        if (p->path != QST_PATH_KRON || p->precision != QST_FP64)
            fail(QST_ERR_UNSUPPORTED, "delayed acceptance uses the FP64 Kronecker path");
    }
}

}  // namespace

extern "C" {

const char* qst_last_error(void) { return g_err.c_str(); }

const char* qst_version(void) { return "qst-gfx950 0.1"; }

qst_status qst_init_problem(const qst_problem_desc* desc, qst_problem** out)
{
    return guarded([&] {
        if (!desc || !out) fail(QST_ERR_INVALID, "NULL argument");
        *out = nullptr;
        const int Q = desc->n_qubits;
        if (Q < 1 || Q > 6) fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
        if (!desc->counts) fail(QST_ERR_INVALID, "counts is NULL");
        if (desc->precision != QST_FP64 && desc->precision != QST_FP32 && desc->precision != QST_BF16X3)
            fail(QST_ERR_INVALID, "unknown precision");
        if (desc->path != QST_PATH_AUTO && desc->path != QST_PATH_DENSE && desc->path != QST_PATH_KRON)
            fail(QST_ERR_INVALID, "unknown path");
        int ndev = 0;
        hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (desc->device < 0 || desc->device >= ndev) fail(QST_ERR_INVALID, "bad device ordinal");
        auto p = std::make_unique<qst_problem>();
        p->Q = Q;
        p->D = 1 << Q;
        p->D2 = p->D * p->D;
        if (desc->param != QST_PARAM_GAMMA && desc->param != QST_PARAM_BURES && desc->param != QST_PARAM_DIRICHLET)
            fail(QST_ERR_INVALID, "unknown parameterisation");
        if (desc->param == QST_PARAM_DIRICHLET && !(desc->alpha > 0.0 && std::isfinite(desc->alpha)))
            fail(QST_ERR_INVALID, "the Dirichlet concentration alpha must be positive and finite");
        p->param = desc->param;
        p->alpha = desc->alpha;
        p->d = p->param == QST_PARAM_BURES ? 4 * p->D2 : 2 * p->D2 + p->D;
        p->K = ipow3(Q);
        p->KD = p->K * p->D;
        p->device = desc->device;
        p->precision = desc->precision;
        p->path = desc->path == QST_PATH_AUTO ? g_auto_path[Q][desc->precision] : desc->path;
        if (p->path == QST_PATH_KRON && p->precision == QST_BF16X3)
            fail(QST_ERR_UNSUPPORTED, "the Kronecker path runs in FP64 or FP32; BF16x3 needs QST_PATH_DENSE");
        if (p->path == QST_PATH_DENSE && Q > 4)
            fail(QST_ERR_UNSUPPORTED,
                 "the dense chain step is built for 1..4 qubits (16 chains of a workgroup share the MFMA tiles, "
                 "and at 5 qubits their states do not fit in LDS); qst_loglik takes QST_PATH_DENSE up to 5 qubits");
        if (desc->povm) {
            // user POVM elements: the dense contraction against their matrix
            if (desc->n_povm < 1 || desc->n_povm > p->KD)
                fail(QST_ERR_INVALID, "n_povm must be in 1..3^Q 2^Q");
            if (desc->path == QST_PATH_KRON)
                fail(QST_ERR_UNSUPPORTED, "user POVMs need the dense path (the Kronecker route is for Pauli settings)");
            if (desc->precision == QST_BF16X3)
                fail(QST_ERR_UNSUPPORTED, "user POVMs run in FP64 or FP32 (BF16x3 needs a matrix exact in BF16)");
            if (Q > 4) fail(QST_ERR_UNSUPPORTED, "dense contraction is built for 1..4 qubits only");
            p->path = QST_PATH_DENSE;
        }
        if (p->param == QST_PARAM_BURES && (p->path != QST_PATH_KRON || Q > 4))
            fail(QST_ERR_UNSUPPORTED, "Algorithm 1 (QST_PARAM_BURES) runs on the Kronecker path, 1..4 qubits");
        if (p->param == QST_PARAM_DIRICHLET && p->path != QST_PATH_KRON)
            fail(QST_ERR_UNSUPPORTED, "Dirichlet weights (QST_PARAM_DIRICHLET) run on the Kronecker path");
        if (desc->povm) {
            p->povm_M = povm_matrix_packed(Q, desc->povm, desc->n_povm);
            p->counts.assign(p->KD, 0);
            std::copy(desc->counts, desc->counts + desc->n_povm, p->counts.begin());
        } else {
            p->counts.assign(desc->counts, desc->counts + p->KD);
        }
        std::vector<double> nd(p->KD);
        for (int i = 0; i < p->KD; ++i) {
            if (p->counts[i] < 0) fail(QST_ERR_INVALID, "negative count");
            nd[i] = static_cast<double>(p->counts[i]);
        }
        std::vector<double> weights;
        if (desc->intensity) {
            const int n_int = desc->povm ? desc->n_povm : p->KD;
            for (int i = 0; i < n_int; ++i)
                if (!(desc->intensity[i] >= 0.0) || !std::isfinite(desc->intensity[i]))
                    fail(QST_ERR_INVALID, "intensities must be finite and >= 0");
            weights = linear_weights_packed(Q, desc->intensity, n_int, p->povm_M);
            p->poisson = true;
        }
        DeviceGuard g(p->device);
        (void)scratch_address(p->device);   // set-up of the allocation-free pooling call
        const size_t nd_len = static_cast<size_t>(p->KD) + weights.size();
        p->nd = dev_alloc<double>(nd_len);
        hip_check(hipMemcpy(p->nd, nd.data(), sizeof(double) * p->KD, hipMemcpyHostToDevice), "copy counts");
        if (!weights.empty())
            hip_check(hipMemcpy(p->nd + p->KD, weights.data(), sizeof(double) * weights.size(), hipMemcpyHostToDevice),
                      "copy Poisson weights");
        // mu(k, t) = sum_q [t_q] (s_q(k) + 1) 4^(Q-1-q): the Pauli string whose
        // coefficient enters position t of setting k's Walsh-Hadamard transform
        std::vector<uint16_t> mu(p->KD);
        for (int k = 0; k < p->K; ++k)
            for (int t = 0; t < p->D; ++t) {
                int m = 0, kk = k;
                for (int q = Q - 1; q >= 0; --q) {
                    const int digit = kk % 3;
                    kk /= 3;
                    if ((t >> (Q - 1 - q)) & 1) m += (digit + 1) << (2 * (Q - 1 - q));
                }
                mu[static_cast<size_t>(k) * p->D + t] = static_cast<uint16_t>(m);
            }
        p->mu = dev_alloc<uint16_t>(p->KD);
        hip_check(hipMemcpy(p->mu, mu.data(), sizeof(uint16_t) * p->KD, hipMemcpyHostToDevice), "copy Pauli index");
        // task-major copies: task u = k L + tl holds positions t = tl + L j,
        // j < V, of setting k (V = min(4, D), L = D / V), entry u V + j
        {
            const int V = p->D < 4 ? p->D : 4, L = p->D / V;
            std::vector<double> ndv(p->KD);
            std::vector<uint16_t> muv(p->KD);
            for (int k = 0; k < p->K; ++k)
                for (int tl = 0; tl < L; ++tl)
                    for (int j = 0; j < V; ++j) {
                        const size_t src = static_cast<size_t>(k) * p->D + tl + L * j;
                        const size_t dst = (static_cast<size_t>(k) * L + tl) * V + j;
                        ndv[dst] = nd[src];
                        muv[dst] = mu[src];
                    }
            p->ndv = dev_alloc<double>(p->KD);
            p->muv = dev_alloc<uint16_t>(p->KD);
            hip_check(hipMemcpy(p->ndv, ndv.data(), sizeof(double) * p->KD, hipMemcpyHostToDevice), "copy counts");
            hip_check(hipMemcpy(p->muv, muv.data(), sizeof(uint16_t) * p->KD, hipMemcpyHostToDevice),
                      "copy Pauli index");
        }
        if (p->path == QST_PATH_DENSE) p->fragments(p->precision);
        *out = p.release();
    });
}

void qst_free_problem(qst_problem* p)
{
    if (!p) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    if (p->last_stream) (void)hipStreamSynchronize(p->last_stream);
    p->free_state();
    dev_free(p->nd);
    dev_free(p->mu);
    dev_free(p->ndv);
    dev_free(p->muv);
    for (auto& f : p->mfrag) dev_free(f);
    (void)hipSetDevice(prev);
    delete p;
}

}  // extern "C"

namespace {

void launch_da(qst_problem* p, const qst_run_desc& r, hipStream_t s);   // delayed acceptance (below)

void prepare_state(qst_problem* p, const qst_run_desc& r)
{
    if (!r.resume) {
        if (p->R != r.n_chains) {
            if (p->last_stream) hip_check(hipStreamSynchronize(p->last_stream), "sync before realloc");
            p->alloc_state(r.n_chains);
        }
        p->step = 0;
        p->chain0 = r.chain_offset;
    }
}

template <typename T>
T* rows_back(T* ptr, int64_t rows, int64_t width)
{
    // ptr moved back by `rows` rows of `width` elements (integer arithmetic:
    // the kernels only touch rows chain0 and later, inside the buffer)
    if (!ptr) return ptr;
    return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(ptr) -
                                static_cast<uintptr_t>(rows) * static_cast<uintptr_t>(width) * sizeof(T));
}

// Arguments of the chain kernels.  problem_wide (the chain and batch
// kernels): chains are addressed by their index within the problem, c in
// [chain_offset, chain_offset + R), and every per-chain buffer is passed
// shifted back by chain_offset rows; otherwise (delayed acceptance) local
// indices in [0, R).
qst::ChainArgs make_args(qst_problem* p, const qst_run_desc& r, bool problem_wide = true)
{
    qst::ChainArgs a{};
    a.nd = p->nd;
    a.mu = p->mu;
    a.ndv = p->ndv;
    a.muv = p->muv;
    a.mfrag = p->path == QST_PATH_DENSE ? p->fragments(p->precision) : nullptr;
    a.R = p->R;
    a.x = p->x;
    a.ll = p->ll;
    a.beta = p->beta;
    a.acc_win = p->accw;
    a.rho_cur = p->rho;
    a.s1 = p->s1;
    a.s2 = p->s2;
    a.n_stored = p->nst;
    a.alpha = p->alpha;
    a.lg_alpha = p->param == QST_PARAM_DIRICHLET ? std::lgamma(p->alpha) : 0.0;
    a.n_acc = p->nacc;
    a.n_near = p->nnear;
    a.step_begin = p->step;
    a.n_steps = r.n_steps;
    a.burn_in = r.burn_in;
    a.adapt_until = r.adapt_until;
    a.thin = r.thin;
    a.adapt_every = r.adapt_every;
    a.init = r.resume ? 0 : 1;
    a.poisson = p->poisson ? 1 : 0;
    a.beta0 = r.beta0;
    a.adapt_lo = r.adapt_lo;
    a.adapt_hi = r.adapt_hi;
    a.adapt_factor = r.adapt_factor;
    a.seed = r.seed;
    a.trace_chains = r.trace_chains;
    a.tr_ll = r.trace_llprop;
    a.tr_lu = r.trace_logu;
    a.tr_acc = r.trace_accept;
    a.record_every = r.record_every;
    a.record_chains = r.record_chains;
    a.rec = r.record_buf;
    a.pair_every = r.pair_every;
    a.pair_chains = r.pair_chains;
    a.pair_width = p->da_width();
    a.pair_x = r.pair_x;
    a.pair_ll = r.pair_ll;
    if (problem_wide && p->chain0 != 0) {
        const int64_t g = p->chain0;
        const int64_t n_rec = r.record_every > 0 ? r.n_steps / r.record_every : 0;
        a.R = g + p->R;
        a.x = rows_back(a.x, g, p->d);
        a.ll = rows_back(a.ll, g, 1);
        a.beta = rows_back(a.beta, g, 1);
        a.acc_win = rows_back(a.acc_win, g, 1);
        a.rho_cur = rows_back(a.rho_cur, g, p->D2);
        a.s1 = rows_back(a.s1, g, p->D2);
        a.s2 = rows_back(a.s2, g, p->D2);
        a.n_stored = rows_back(a.n_stored, g, 1);
        a.n_acc = rows_back(a.n_acc, g, 1);
        a.n_near = rows_back(a.n_near, g, 1);
        a.trace_chains = static_cast<int32_t>(g + r.trace_chains);
        a.tr_ll = rows_back(a.tr_ll, g, r.n_steps);
        a.tr_lu = rows_back(a.tr_lu, g, r.n_steps);
        a.tr_acc = rows_back(a.tr_acc, g, r.n_steps);
        a.record_chains = static_cast<int32_t>(g + r.record_chains);
        a.rec = rows_back(a.rec, g, n_rec * p->D2);
        // the pair recorder runs with chain_offset 0 (validate_run)
    }
    return a;
}

qst_run_stats collect_stats(const qst_problem* p, const qst_run_desc& r)
{
    std::vector<int64_t> nacc(p->R), nnear(p->R);
    std::vector<double> ll(p->R), beta(p->R);
    hip_check(hipMemcpy(nacc.data(), p->nacc, sizeof(int64_t) * p->R, hipMemcpyDeviceToHost), "stats");
    hip_check(hipMemcpy(nnear.data(), p->nnear, sizeof(int64_t) * p->R, hipMemcpyDeviceToHost), "stats");
    hip_check(hipMemcpy(ll.data(), p->ll, sizeof(double) * p->R, hipMemcpyDeviceToHost), "stats");
    hip_check(hipMemcpy(beta.data(), p->beta, sizeof(double) * p->R, hipMemcpyDeviceToHost), "stats");
    qst_run_stats st{};
    st.proposed = p->R * r.n_steps;
    st.beta_min = INFINITY;
    st.beta_max = -INFINITY;
    for (int64_t c = 0; c < p->R; ++c) {
        st.accepted += nacc[c];
        st.near_threshold += nnear[c];
        st.nonfinite_chains += std::isfinite(ll[c]) ? 0 : 1;
        st.beta_min = std::fmin(st.beta_min, beta[c]);
        st.beta_max = std::fmax(st.beta_max, beta[c]);
    }
    st.stage1_passed = st.proposed;
    return st;
}

int batch_team(int Q)
{
    switch (Q) {
        case 1: return qst::BatchTeam<1>::G;
        case 2: return qst::BatchTeam<2>::G;
        case 3: return qst::BatchTeam<3>::G;
        case 4: return qst::BatchTeam<4>::G;
        case 5: return qst::BatchTeam<5>::G;
        default: return qst::BatchTeam<6>::G;
    }
}

size_t batch_lds_bytes(int Q)
{
    switch (Q) {
        case 1: return qst::batch_lds_doubles<1>() * sizeof(double);
        case 2: return qst::batch_lds_doubles<2>() * sizeof(double);
        case 3: return qst::batch_lds_doubles<3>() * sizeof(double);
        case 4: return qst::batch_lds_doubles<4>() * sizeof(double);
        case 5: return qst::batch_lds_doubles<5>() * sizeof(double);
        default: return qst::batch_lds_doubles<6>() * sizeof(double);
    }
}

// Cost of one chain-step per qubit count for the largest-first ordering of
// batch tiles (ns of a full MI355X per chain-step, measured with the tuned
// shapes; only the order matters).
double chain_step_cost(int Q)
{
    static const double c[7] = {0.0, 0.16, 0.37, 1.6, 5.2, 32.0, 320.0};
    return c[Q];
}

// Worker streams of the uneven batch, per device: created once at the
// default priority and kept for the process, so that the launch classes of a
// batch run side by side instead of back to back.
constexpr int kBatchStreams = 4;

hipStream_t* batch_streams(int dev)
{
    static std::mutex mu;
    static std::map<int, std::vector<hipStream_t>> streams;
    std::lock_guard<std::mutex> lock(mu);
    std::vector<hipStream_t>& v = streams[dev];
    while (v.size() < static_cast<size_t>(kBatchStreams)) {
        hipStream_t st = nullptr;
        hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "batch stream");
        v.push_back(st);
    }
    return v.data();
}

// One persistent launch per qubit count and precision over its part of the
// tile list (n tiles from `items`, largest first) with its own counter.
template <int QMAX, int PREC>
void launch_batch_class(const qst::BatchItem* items, size_t n, size_t lds, const qst::ChainArgs* dargs,
                        int32_t* counter, int n_cu, hipStream_t s)
{
    if (n == 0) return;
    qst::BatchArgs b{dargs, items, static_cast<int32_t>(n), counter};
    if constexpr (QMAX == 6) {   // one workgroup per tile (batch_kernel.hpp)
        allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_chains_batch_grid<QMAX, PREC>), lds);
        hipLaunchKernelGGL((qst::k_chains_batch_grid<QMAX, PREC>), dim3(static_cast<unsigned>(n)),
                           dim3(qst::batch_wg(QMAX)), lds, s, b);
        hip_check(hipGetLastError(), "batch kernel launch");
        return;
    }
    allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_chains_batch<QMAX, PREC>), lds);
    int per_cu = 0;
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, qst::k_chains_batch<QMAX, PREC>,
                                                           qst::batch_wg(QMAX), lds),
              "occupancy");
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(static_cast<int64_t>(n),
                                                                 static_cast<int64_t>(n_cu) * std::max(per_cu, 1)));
    hipLaunchKernelGGL((qst::k_chains_batch<QMAX, PREC>), dim3(static_cast<unsigned>(grid)),
                       dim3(qst::batch_wg(QMAX)), lds, s, b);
    hip_check(hipGetLastError(), "batch kernel launch");
}

void launch_batch(qst_problem* const* problems, int32_t n, const qst_run_desc* runs, hipStream_t s)
{
    std::vector<qst::ChainArgs> args(n);
    std::vector<qst::BatchItem> items;
    std::vector<double> cost;
    size_t lds_class[7] = {0, 0, 0, 0, 0, 0, 0};   // by qubit count
    for (int i = 0; i < n; ++i) {
        qst_problem* p = problems[i];
        if (p->path != QST_PATH_KRON)
            fail(QST_ERR_UNSUPPORTED,
                 "batched launches use the Kronecker path (FP64 or FP32): the dense forms run only to 4 qubits, "
                 "each at a fraction of the Kronecker route's rate, and need 16-chain workgroups of their own");
        args[i] = make_args(p, runs[i]);
        const int per = qst::batch_wg(qst::batch_class(p->Q)) / batch_team(p->Q);
        const int32_t prec = p->precision == QST_FP32 ? qst::kPrecF32 : qst::kPrecF64;
        for (int64_t c0 = 0; c0 < p->R; c0 += per) {
            items.push_back({i, p->Q, p->chain0 + c0, prec, 0});   // problem-wide chain index (make_args)
            cost.push_back(chain_step_cost(p->Q) * static_cast<double>(std::min<int64_t>(per, p->R - c0)) *
                           static_cast<double>(std::max<int64_t>(runs[i].n_steps, 1)));
        }
        size_t& l = lds_class[qst::batch_class(p->Q)];
        l = std::max(l, batch_lds_bytes(p->Q));
    }
    std::vector<size_t> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    // one list: the classes in launch order (6 qubits first, FP64 before
    // FP32), each largest first
    constexpr int kClasses = 12;
    auto slot = [](int q, int prec) { return 2 * (6 - q) + prec; };
    std::vector<qst::BatchItem> by_slot[kClasses];
    for (size_t i : order) by_slot[slot(items[i].q, items[i].prec)].push_back(items[i]);
    std::vector<qst::BatchItem> all;
    size_t off[kClasses + 1] = {};
    for (int k = 0; k < kClasses; ++k) {
        off[k] = all.size();
        all.insert(all.end(), by_slot[k].begin(), by_slot[k].end());
    }
    off[kClasses] = all.size();
    for (int k = 0; k < kClasses; ++k)
        if (off[k + 1] - off[k] > 0x7fffffff) fail(QST_ERR_INVALID, "batch too large");

    qst::ChainArgs* dargs = dev_alloc<qst::ChainArgs>(args.size());
    qst::BatchItem* ditems = nullptr;
    int32_t* counters = nullptr;
    try {
        ditems = dev_alloc<qst::BatchItem>(std::max<size_t>(1, all.size()));
        counters = dev_alloc<int32_t>(kClasses);
        hip_check(hipMemcpy(dargs, args.data(), sizeof(qst::ChainArgs) * args.size(), hipMemcpyHostToDevice),
                  "copy batch problems");
        hip_check(hipMemcpy(ditems, all.data(), sizeof(qst::BatchItem) * all.size(), hipMemcpyHostToDevice),
                  "copy batch tiles");
        int dev = 0, n_cu = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        hip_check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
        hipLaunchKernelGGL(qst::k_zero_counters, dim3(1), dim3(64), 0, s, counters, kClasses);
        hip_check(hipGetLastError(), "counter reset");
        // the classes go round-robin onto the worker streams, largest qubit
        // count first, each stream starting after the work already on s;
        // whatever CUs a class leaves idle while it drains, the next class
        // on another stream fills
        hipStream_t* ws = batch_streams(dev);
        hipEvent_t start = nullptr, done[kBatchStreams] = {};
        hip_check(hipEventCreateWithFlags(&start, hipEventDisableTiming), "batch event");
        for (auto& e : done) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "batch event");
        hip_check(hipEventRecord(start, s), "batch event record");
        for (int i = 0; i < kBatchStreams; ++i) hip_check(hipStreamWaitEvent(ws[i], start, 0), "batch stream wait");
        int next = 0;
        bool used[kBatchStreams] = {};
        constexpr int F64 = qst::kPrecF64, F32 = qst::kPrecF32;
        auto both = [&](auto qc) {
            constexpr int Q = decltype(qc)::value;
            const int k64 = slot(Q, F64), k32 = slot(Q, F32);
            for (int k : {k64, k32}) {
                if (off[k + 1] == off[k]) continue;
                const int si = next++ % kBatchStreams;
                used[si] = true;
                if (k == k64)
                    launch_batch_class<Q, F64>(ditems + off[k], off[k + 1] - off[k], lds_class[Q], dargs,
                                               counters + k, n_cu, ws[si]);
                else
                    launch_batch_class<Q, F32>(ditems + off[k], off[k + 1] - off[k], lds_class[Q], dargs,
                                               counters + k, n_cu, ws[si]);
            }
        };
        both(std::integral_constant<int, 6>{});
        both(std::integral_constant<int, 5>{});
        both(std::integral_constant<int, 4>{});
        both(std::integral_constant<int, 3>{});
        both(std::integral_constant<int, 2>{});
        both(std::integral_constant<int, 1>{});
        for (int i = 0; i < kBatchStreams; ++i) {
            if (!used[i]) continue;
            hip_check(hipEventRecord(done[i], ws[i]), "batch event record");
            hip_check(hipStreamWaitEvent(s, done[i], 0), "batch join");
        }
        hip_check(hipStreamSynchronize(s), "batch synchronize");
        (void)hipEventDestroy(start);
        for (auto& e : done) (void)hipEventDestroy(e);
    } catch (...) {
        (void)hipDeviceSynchronize();    // no launch, on s or a worker stream, may still read the buffers freed below
        dev_free(dargs);
        dev_free(ditems);
        dev_free(counters);
        throw;
    }
    dev_free(dargs);
    dev_free(ditems);
    dev_free(counters);
}

}  // namespace

extern "C" {

qst_status qst_run_chains(qst_problem* const* problems, int32_t n_problems, const qst_run_desc* runs,
                          qst_run_stats* stats)
{
    return guarded([&] {
        if (!problems || !runs || n_problems < 1) fail(QST_ERR_INVALID, "empty batch");
        const int dev = problems[0] ? problems[0]->device : 0;
        for (int i = 0; i < n_problems; ++i) {
            if (!problems[i]) fail(QST_ERR_INVALID, "NULL problem handle");
            if (problems[i]->device != dev) fail(QST_ERR_INVALID, "batch spans several devices");
            for (int j = 0; j < i; ++j)
                if (problems[j] == problems[i]) fail(QST_ERR_INVALID, "a handle appears twice in the batch");
            validate_run(problems[i], runs[i]);
            if (n_problems > 1 && problems[i]->param != QST_PARAM_GAMMA)
                fail(QST_ERR_UNSUPPORTED, "batches run the Gaussian/gamma parameterisation");
        }
        DeviceGuard g(dev);
        hipStream_t s = static_cast<hipStream_t>(runs[0].stream);
        for (int i = 0; i < n_problems; ++i) prepare_state(problems[i], runs[i]);
        // states set by qst_set_chain_state: log L and packed rho evaluated by
        // the restore kernel of the same shape and code, then the run resumes
        // from them
        for (int i = 0; i < n_problems; ++i) {
            qst_problem* p = problems[i];
            if (!p->reeval) continue;
            if (runs[i].resume) {
                qst_run_desc r0 = runs[i];
                r0.n_steps = 0;
                r0.surrogate = nullptr;
                r0.trace_chains = 0;
                r0.record_every = r0.record_chains = 0;
                r0.pair_every = r0.pair_chains = 0;
                const qst::ChainArgs a0 = make_args(p, r0);
                if (p->param == QST_PARAM_BURES)
                    launch_chains_bures(p->Q, static_cast<int>(p->precision), a0, p->chain0, s, true);
                else if (p->param == QST_PARAM_DIRICHLET)
                    launch_chains_dirichlet(p->Q, static_cast<int>(p->precision), a0, p->chain0, s, true);
                else
                    launch_chains(p->Q, current_shape(p->Q),
                                  p->path == QST_PATH_DENSE ? qst::kPathDense : qst::kPathKron,
                                  static_cast<int>(p->precision), a0, p->chain0, s, true);
            }
            p->reeval = false;
        }
        if (n_problems == 1 && runs[0].surrogate) {
            launch_da(problems[0], runs[0], s);
        } else if (n_problems == 1) {
            qst_problem* p = problems[0];
            const qst::ChainArgs a = make_args(p, runs[0]);
            if (p->param == QST_PARAM_BURES)
                launch_chains_bures(p->Q, static_cast<int>(p->precision), a, p->chain0, s);
            else if (p->param == QST_PARAM_DIRICHLET)
                launch_chains_dirichlet(p->Q, static_cast<int>(p->precision), a, p->chain0, s);
            else
                launch_chains(p->Q, current_shape(p->Q), p->path == QST_PATH_DENSE ? qst::kPathDense : qst::kPathKron,
                              static_cast<int>(p->precision), a, p->chain0, s);
        } else {
            for (int i = 0; i < n_problems; ++i)
                if (runs[i].surrogate)
                    fail(QST_ERR_UNSUPPORTED, "delayed acceptance runs one problem per call: each of its steps is "
                                              "four launches (propose, network, screen, exact stage) with the "
                                              "chain state in HBM, not a persistent tile");
            launch_batch(problems, n_problems, runs, s);
        }
        for (int i = 0; i < n_problems; ++i) {
            problems[i]->step += runs[i].n_steps;
            problems[i]->have_run = true;
            problems[i]->last_stream = s;
        }
        if (stats) {
            hip_check(hipStreamSynchronize(s), "run synchronize");
            for (int i = 0; i < n_problems; ++i) {
                stats[i] = collect_stats(problems[i], runs[i]);
                if (runs[i].surrogate) {
                    std::vector<int64_t> s1(problems[i]->R);
                    hip_check(hipMemcpy(s1.data(), problems[i]->n_stage1, sizeof(int64_t) * s1.size(),
                                        hipMemcpyDeviceToHost), "stats");
                    int64_t tot = 0;
                    for (int64_t v : s1) tot += v;
                    stats[i].stage1_passed = tot;
                }
            }
        }
    });
}

qst_status qst_set_launch_shape(int32_t n_qubits, int32_t team, int32_t workgroup)
{
    return guarded([&] {
        if (n_qubits < 1 || n_qubits > 6) fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
        const Shape sh{team, workgroup};
        if (!shape_compiled(n_qubits, sh)) fail(QST_ERR_UNSUPPORTED, "no chain kernel compiled for this shape");
        g_shape[n_qubits] = sh;
    });
}

qst_status qst_set_auto_path(int32_t n_qubits, qst_precision precision, qst_path path)
{
    return guarded([&] {
        if (n_qubits < 1 || n_qubits > 6) fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
        if (precision != QST_FP64 && precision != QST_FP32 && precision != QST_BF16X3)
            fail(QST_ERR_INVALID, "unknown precision");
        if (path != QST_PATH_DENSE && path != QST_PATH_KRON) fail(QST_ERR_INVALID, "path must be DENSE or KRON");
        if (path == QST_PATH_KRON && precision == QST_BF16X3)
            fail(QST_ERR_UNSUPPORTED, "the Kronecker path runs in FP64 or FP32");
        if (path == QST_PATH_DENSE && n_qubits > 4) fail(QST_ERR_UNSUPPORTED, "the dense chain step stops at 4 qubits");
        g_auto_path[n_qubits][precision] = path;
    });
}

qst_status qst_get_auto_path(int32_t n_qubits, qst_precision precision, qst_path* path)
{
    return guarded([&] {
        if (n_qubits < 1 || n_qubits > 6 || !path) fail(QST_ERR_INVALID, "bad argument");
        if (precision != QST_FP64 && precision != QST_FP32 && precision != QST_BF16X3)
            fail(QST_ERR_INVALID, "unknown precision");
        *path = g_auto_path[n_qubits][precision];
    });
}

qst_status qst_get_launch_shape(int32_t n_qubits, int32_t* team, int32_t* workgroup)
{
    return guarded([&] {
        if (n_qubits < 1 || n_qubits > 6) fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
        if (!team || !workgroup) fail(QST_ERR_INVALID, "NULL output");
        *team = g_shape[n_qubits].G;
        *workgroup = g_shape[n_qubits].WG;
    });
}

qst_status qst_get_batch_shape(int32_t n_qubits, int32_t* team, int32_t* workgroup)
{
    return guarded([&] {
        if (n_qubits < 1 || n_qubits > 6) fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
        if (!team || !workgroup) fail(QST_ERR_INVALID, "NULL output");
        *team = batch_team(n_qubits);
        *workgroup = qst::batch_wg(qst::batch_class(n_qubits));
    });
}

qst_status qst_list_launch_shapes(int32_t n_qubits, int32_t* teams, int32_t* workgroups, int32_t capacity,
                                  int32_t* count)
{
    return guarded([&] {
        if (n_qubits < 1 || n_qubits > 6) fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
        if (!count) fail(QST_ERR_INVALID, "NULL count");
        int32_t n = 0;
        for (const Shape& c : kShapes[n_qubits]) {
            if (c.G <= 0) continue;
            if (teams && workgroups && n < capacity) {
                teams[n] = c.G;
                workgroups[n] = c.WG;
            }
            ++n;
        }
        *count = n;
    });
}

qst_status qst_pool_moments(const qst_problem* p, double* mean, double* second, double* se, int64_t* n_samples)
{
    return guarded([&] {
        if (!p) fail(QST_ERR_INVALID, "NULL handle");
        if (!p->have_run) fail(QST_ERR_STATE, "pool before any run");
        if (!mean) fail(QST_ERR_INVALID, "mean is NULL");
        DeviceGuard g(p->device);
        hipStream_t s = p->last_stream;
        const int64_t chunk = 256;
        const int nchunks = static_cast<int>((p->R + chunk - 1) / chunk);
        double* part = dev_alloc<double>(static_cast<size_t>(nchunks) * 5 * p->D2);
        int64_t* nsum = nullptr;
        double* outd = nullptr;
        int64_t* nout = nullptr;
        try {
            nsum = dev_alloc<int64_t>(nchunks);
            outd = dev_alloc<double>(static_cast<size_t>(6) * p->D2);
            nout = dev_alloc<int64_t>(1);
            hipLaunchKernelGGL(qst::k_pool_partial, dim3(nchunks), dim3(qst::kPoolThreads), 0, s, p->s1, p->s2,
                               p->nst, p->R, p->D2, chunk, part, nsum);
            hip_check(hipGetLastError(), "pool partial launch");
            hipLaunchKernelGGL(qst::k_pool_final, dim3((p->D2 + qst::kPoolThreads - 1) / qst::kPoolThreads),
                               dim3(qst::kPoolThreads), 0, s, part, nsum, nchunks, p->D, outd, nout);
            hip_check(hipGetLastError(), "pool final launch");
            std::vector<double> host(static_cast<size_t>(6) * p->D2);
            int64_t ntot = 0;
            hip_check(hipStreamSynchronize(s), "pool synchronize");
            hip_check(hipMemcpy(host.data(), outd, sizeof(double) * host.size(), hipMemcpyDeviceToHost), "pool copy");
            hip_check(hipMemcpy(&ntot, nout, sizeof(int64_t), hipMemcpyDeviceToHost), "pool copy");
            if (ntot == 0) fail(QST_ERR_STATE, "no stored samples (burn_in/thin exclude every step)");
            std::memcpy(mean, host.data(), sizeof(double) * 2 * p->D2);
            if (second) std::memcpy(second, host.data() + 2 * p->D2, sizeof(double) * 2 * p->D2);
            if (se) std::memcpy(se, host.data() + 4 * p->D2, sizeof(double) * 2 * p->D2);
            if (n_samples) *n_samples = ntot;
        } catch (...) {
            dev_free(part);
            dev_free(nsum);
            dev_free(outd);
            dev_free(nout);
            throw;
        }
        dev_free(part);
        dev_free(nsum);
        dev_free(outd);
        dev_free(nout);
    });
}

qst_status qst_pool_moments_static(const qst_problem* p, double* out, int64_t* n_out, void* stream)
{
    return guarded([&] {
        if (!p) fail(QST_ERR_INVALID, "NULL handle");
        if (!p->have_run) fail(QST_ERR_STATE, "pool before any run");
        if (!out || !n_out) fail(QST_ERR_INVALID, "NULL output");
        const int64_t chunk = 256;
        const int64_t nchunks = (p->R + chunk - 1) / chunk;
        const size_t part_doubles = static_cast<size_t>(nchunks) * 5 * p->D2;
        // partial sums, then the per-chunk sample counts at the next 256-byte boundary
        const size_t nsum_off = (part_doubles * sizeof(double) + 255) / 256 * 256;
        const size_t need = nsum_off + static_cast<size_t>(nchunks) * sizeof(int64_t);
        if (need > kScratchBytes)
            fail(QST_ERR_INVALID, "pooling " + std::to_string(p->R) + " chains of " + std::to_string(p->Q) +
                                      " qubits needs " + std::to_string(need) + " bytes of scratch; the static "
                                      "scratch holds " + std::to_string(kScratchBytes) +
                                      " (use qst_pool_moments)");
        check_device_buffer(out, static_cast<size_t>(6) * p->D2 * sizeof(double), p->device, "out");
        check_device_buffer(n_out, sizeof(int64_t), p->device, "n_out");
        DeviceGuard g(p->device);
        char* base = static_cast<char*>(scratch_address(p->device));
        double* part = reinterpret_cast<double*>(base);
        int64_t* nsum = reinterpret_cast<int64_t*>(base + nsum_off);
        hipStream_t s = static_cast<hipStream_t>(stream);
        // both passes write every scratch entry they read: nothing to clear
        hipLaunchKernelGGL(qst::k_pool_partial, dim3(static_cast<unsigned>(nchunks)), dim3(qst::kPoolThreads), 0, s,
                           p->s1, p->s2, p->nst, p->R, p->D2, chunk, part, nsum);
        hip_check(hipGetLastError(), "pool partial launch");
        hipLaunchKernelGGL(qst::k_pool_final, dim3((p->D2 + qst::kPoolThreads - 1) / qst::kPoolThreads),
                           dim3(qst::kPoolThreads), 0, s, part, nsum, static_cast<int>(nchunks), p->D, out, n_out);
        hip_check(hipGetLastError(), "pool final launch");
    });
}

qst_status qst_chain_state(const qst_problem* p, double* x, double* loglik, double* beta, int64_t* n_stored)
{
    return guarded([&] {
        if (!p) fail(QST_ERR_INVALID, "NULL handle");
        if (!p->have_run) fail(QST_ERR_STATE, "no chains yet");
        DeviceGuard g(p->device);
        if (p->last_stream) hip_check(hipStreamSynchronize(p->last_stream), "state synchronize");
        if (x) hip_check(hipMemcpy(x, p->x, sizeof(double) * p->R * p->d, hipMemcpyDeviceToHost), "state copy");
        if (loglik) hip_check(hipMemcpy(loglik, p->ll, sizeof(double) * p->R, hipMemcpyDeviceToHost), "state copy");
        if (beta) hip_check(hipMemcpy(beta, p->beta, sizeof(double) * p->R, hipMemcpyDeviceToHost), "state copy");
        if (n_stored)
            hip_check(hipMemcpy(n_stored, p->nst, sizeof(int64_t) * p->R, hipMemcpyDeviceToHost), "state copy");
    });
}

qst_status qst_set_chain_state(qst_problem* p, int64_t step, const double* x, const double* beta, const double* s1,
                               const double* s2, const int64_t* n_stored)
{
    return guarded([&] {
        if (!p) fail(QST_ERR_INVALID, "NULL handle");
        if (!p->have_run) fail(QST_ERR_STATE, "no chains yet: run (n_steps 0 allocates and initialises them) first");
        if (step < -1) fail(QST_ERR_INVALID, "step must be >= 0 (or -1 to keep)");
        if (beta)
            for (int64_t c = 0; c < p->R; ++c)
                if (!(beta[c] > 0.0 && beta[c] <= 1.0)) fail(QST_ERR_INVALID, "beta must lie in (0, 1]");
        if (n_stored)
            for (int64_t c = 0; c < p->R; ++c)
                if (n_stored[c] < 0) fail(QST_ERR_INVALID, "n_stored must be >= 0");
        DeviceGuard g(p->device);
        if (p->last_stream) hip_check(hipStreamSynchronize(p->last_stream), "state synchronize");
        const size_t R = static_cast<size_t>(p->R), m = R * p->D2;
        if (x) hip_check(hipMemcpy(p->x, x, sizeof(double) * R * p->d, hipMemcpyHostToDevice), "state copy");
        if (beta) hip_check(hipMemcpy(p->beta, beta, sizeof(double) * R, hipMemcpyHostToDevice), "state copy");
        if (s1) hip_check(hipMemcpy(p->s1, s1, sizeof(double) * m, hipMemcpyHostToDevice), "state copy");
        if (s2) hip_check(hipMemcpy(p->s2, s2, sizeof(double) * m, hipMemcpyHostToDevice), "state copy");
        if (n_stored) hip_check(hipMemcpy(p->nst, n_stored, sizeof(int64_t) * R, hipMemcpyHostToDevice), "state copy");
        if (step >= 0) p->step = step;
        if (x) p->reeval = true;
    });
}

qst_status qst_chain_moments(const qst_problem* p, double* s1, double* s2)
{
    return guarded([&] {
        if (!p) fail(QST_ERR_INVALID, "NULL handle");
        if (!p->have_run) fail(QST_ERR_STATE, "no chains yet");
        DeviceGuard g(p->device);
        if (p->last_stream) hip_check(hipStreamSynchronize(p->last_stream), "moments synchronize");
        const size_t n = static_cast<size_t>(p->R) * p->D2;
        if (s1) hip_check(hipMemcpy(s1, p->s1, sizeof(double) * n, hipMemcpyDeviceToHost), "moments copy");
        if (s2) hip_check(hipMemcpy(s2, p->s2, sizeof(double) * n, hipMemcpyDeviceToHost), "moments copy");
    });
}

qst_status qst_loglik(const qst_problem* p, const double* rho, int64_t n, double* ll_out, qst_path path,
                      qst_precision precision, void* stream)
{
    return guarded([&] {
        if (!p) fail(QST_ERR_INVALID, "NULL handle");
        if (n < 0) fail(QST_ERR_INVALID, "negative n");
        if (n == 0) return;
        if (!rho || !ll_out) fail(QST_ERR_INVALID, "NULL buffer");
        check_device_buffer(rho, static_cast<size_t>(n) * p->D2 * 2 * sizeof(double), p->device, "rho");
        check_device_buffer(ll_out, static_cast<size_t>(n) * sizeof(double), p->device, "ll_out");
        const qst_path pth = path == QST_PATH_AUTO ? p->path : path;
        if (pth == QST_PATH_KRON && !p->povm_M.empty())
            fail(QST_ERR_UNSUPPORTED, "user POVMs need the dense path");
        if (precision == QST_BF16X3 && !p->povm_M.empty())
            fail(QST_ERR_UNSUPPORTED, "user POVMs run in FP64 or FP32");
        if (precision != QST_FP64 && precision != QST_FP32 && precision != QST_BF16X3)
            fail(QST_ERR_INVALID, "unknown precision");
        if (pth == QST_PATH_KRON && precision == QST_BF16X3)
            fail(QST_ERR_UNSUPPORTED, "the Kronecker path runs in FP64 or FP32");
        DeviceGuard g(p->device);
        if (pth == QST_PATH_DENSE) {
            const void* f = const_cast<qst_problem*>(p)->fragments(precision);
            launch_loglik_dense(p->Q, precision, p->nd, f, rho, n, ll_out, p->poisson ? 1 : 0,
                                static_cast<hipStream_t>(stream));
        } else {
            launch_loglik(p->Q, precision == QST_FP32 ? qst::kPrecF32 : qst::kPrecF64, p->nd, p->mu, p->ndv, p->muv,
                          rho, n, ll_out, p->poisson ? 1 : 0, static_cast<hipStream_t>(stream));
        }
    });
}

qst_status qst_acf(const double* records, int64_t n_chains, int64_t n_samples, int32_t n_qubits, int32_t l_max,
                   double* out, void* stream)
{
    return guarded([&] {
        if (!records || !out) fail(QST_ERR_INVALID, "NULL buffer");
        if (n_qubits < 1 || n_qubits > 6) fail(QST_ERR_INVALID, "n_qubits must be in 1..6");
        if (n_chains < 1 || l_max < 0 || n_samples <= l_max)
            fail(QST_ERR_INVALID, "need n_chains >= 1 and n_samples > l_max >= 0");
        if (n_chains > 65535) fail(QST_ERR_INVALID, "at most 65535 recorded chains");
        check_device_buffer(records, static_cast<size_t>(n_chains) * n_samples * (size_t(1) << (2 * n_qubits)) *
                                         sizeof(double), current_device(), "records");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int D = 1 << n_qubits;
        double* part = dev_alloc<double>(static_cast<size_t>(n_chains) * (l_max + 1));
        double* outd = nullptr;
        try {
            outd = dev_alloc<double>(l_max + 1);
            const int n_groups = (l_max + 1 + qst::kAcfLags - 1) / qst::kAcfLags;
            const int64_t blocks = n_chains * n_groups;
            if (blocks > 0x7fffffff) fail(QST_ERR_INVALID, "too many chains x lags");
            hipLaunchKernelGGL(qst::k_acf_partial, dim3(static_cast<unsigned>(blocks)), dim3(qst::kAcfThreads), 0, s,
                               records, n_samples, D, l_max, n_groups, n_chains, part);
            hip_check(hipGetLastError(), "acf launch");
            hipLaunchKernelGGL(qst::k_acf_final, dim3(1), dim3(qst::kAcfThreads), 0, s, part, n_chains, l_max, outd);
            hip_check(hipGetLastError(), "acf final launch");
            hip_check(hipStreamSynchronize(s), "acf synchronize");
            hip_check(hipMemcpy(out, outd, sizeof(double) * (l_max + 1), hipMemcpyDeviceToHost), "acf copy");
        } catch (...) {
            dev_free(part);
            dev_free(outd);
            throw;
        }
        dev_free(part);
        dev_free(outd);
    });
}

}  // extern "C"

// ===========================================================================
// MLP surrogate (delayed acceptance): parameters, workspaces, training step
// ===========================================================================
struct qst_mlp {
    int d = 0, h1 = 0, h2 = 0, device = 0;
    int64_t n_par = 0;
    int64_t t = 0;                 // Adam steps taken
    float out_scale = 1.0f, out_shift = 0.0f;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *W1b = nullptr, *W2b = nullptr, *W2T = nullptr;
    // workspace for batches up to cap rows
    int64_t cap = 0;
    float *Z1 = nullptr, *Z2 = nullptr, *s = nullptr, *ds = nullptr, *sq = nullptr, *part = nullptr, *loss = nullptr;
    uint16_t *H1 = nullptr, *H2 = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *dZ2T = nullptr, *H1T = nullptr,
             *dZ1T = nullptr, *XT = nullptr;

    int64_t off_W1() const { return 0; }
    int64_t off_b1() const { return static_cast<int64_t>(h1) * d; }
    int64_t off_W2() const { return off_b1() + h1; }
    int64_t off_b2() const { return off_W2() + static_cast<int64_t>(h2) * h1; }
    int64_t off_w3() const { return off_b2() + h2; }
    int64_t off_b3() const { return off_w3() + h2; }

    void free_work()
    {
        dev_free(Z1); dev_free(Z2); dev_free(s); dev_free(ds); dev_free(sq); dev_free(part); dev_free(loss);
        dev_free(H1); dev_free(H2); dev_free(dZ2); dev_free(dZ1); dev_free(dZ2T); dev_free(H1T); dev_free(dZ1T);
        dev_free(XT);
        cap = 0;
    }
    void ensure(int64_t n)
    {
        if (n <= cap) return;
        free_work();
        const int64_t c = (n + 63) / 64 * 64;
        const int64_t hmax = std::max(h1, h2);
        Z1 = dev_alloc<float>(c * h1);
        Z2 = dev_alloc<float>(c * h2);
        s = dev_alloc<float>(c);
        ds = dev_alloc<float>(c);
        sq = dev_alloc<float>(c);
        part = dev_alloc<float>(((c + qst::kColChunk - 1) / qst::kColChunk) * std::max<int64_t>(hmax, 1));
        loss = dev_alloc<float>(1);
        H1 = dev_alloc<uint16_t>(c * h1);
        H2 = dev_alloc<uint16_t>(c * h2);
        dZ2 = dev_alloc<uint16_t>(c * h2);
        dZ1 = dev_alloc<uint16_t>(c * h1);
        dZ2T = dev_alloc<uint16_t>(c * h2);
        H1T = dev_alloc<uint16_t>(c * h1);
        dZ1T = dev_alloc<uint16_t>(c * h1);
        XT = dev_alloc<uint16_t>(c * d);
        cap = c;
    }
    void free_all()
    {
        free_work();
        dev_free(theta); dev_free(grad); dev_free(m); dev_free(v); dev_free(W1b); dev_free(W2b); dev_free(W2T);
    }
};

namespace {

inline unsigned blocks_for(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

void mlp_refresh_bf16(qst_mlp* h, hipStream_t s)
{
    const int64_t n1 = static_cast<int64_t>(h->h1) * h->d, n2 = static_cast<int64_t>(h->h2) * h->h1;
    hipLaunchKernelGGL(qst::k_f32_to_bf16, dim3(blocks_for(n1, 256)), dim3(256), 0, s, h->theta + h->off_W1(), n1, h->W1b);
    hipLaunchKernelGGL(qst::k_f32_to_bf16, dim3(blocks_for(n2, 256)), dim3(256), 0, s, h->theta + h->off_W2(), n2, h->W2b);
    hip_check(hipGetLastError(), "weight conversion");
}

template <int EPI>
void gemm(int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C, int ldc,
          const float* bias, const float* Zin, float* Zout, uint16_t* H, int ldh, hipStream_t s)
{
    if (K % qst::kMlpBK != 0) fail(QST_ERR_INVALID, "product length must be a multiple of 32");
    const dim3 grid(blocks_for(N, qst::kMlpTile), blocks_for(M, qst::kMlpTile));
    hipLaunchKernelGGL((qst::k_gemm_nt_bf16<EPI>), grid, dim3(256), 0, s, M, N, A, lda, B, ldb, K, C, ldc, bias, Zin,
                       Zout, H, ldh);
    hip_check(hipGetLastError(), "MLP product launch");
}

void colsum(const uint16_t* in, const float* w, int64_t rows, int cols, float* part, float* out, hipStream_t s)
{
    const int nchunks = static_cast<int>((rows + qst::kColChunk - 1) / qst::kColChunk);
    hipLaunchKernelGGL(qst::k_colsum_partial, dim3(blocks_for(cols, 256), nchunks), dim3(256), 0, s, in, w, rows, cols,
                       part);
    hipLaunchKernelGGL(qst::k_colsum_final, dim3(blocks_for(cols, 256)), dim3(256), 0, s, part, nchunks, cols, out);
    hip_check(hipGetLastError(), "column sum launch");
}

// forward of n rows of X (BF16 [n][d]); s_out (nullable) gets scale*s + shift;
// with y, the loss pieces (ds, sq) too
void mlp_forward(qst_mlp* h, const uint16_t* X, int64_t n, float* s_out, const float* y, hipStream_t s)
{
    h->ensure(n);
    const int N = static_cast<int>(n);
    gemm<qst::kBiasGelu>(N, h->h1, h->d, X, h->d, h->W1b, h->d, nullptr, h->h1, h->theta + h->off_b1(), nullptr, h->Z1,
                         h->H1, h->h1, s);
    gemm<qst::kBiasGelu>(N, h->h2, h->h1, h->H1, h->h1, h->W2b, h->h1, nullptr, h->h2, h->theta + h->off_b2(), nullptr,
                         h->Z2, h->H2, h->h2, s);
    hipLaunchKernelGGL(qst::k_last_fwd, dim3(blocks_for(n, 4)), dim3(256), 0, s, h->H2, h->h2, h->theta + h->off_w3(),
                       h->theta + h->off_b3(), n, h->out_scale, h->out_shift, s_out, y, h->ds, h->sq);
    hip_check(hipGetLastError(), "last layer launch");
}

// gradients of the mean squared error into h->grad, loss into h->loss
void mlp_backward(qst_mlp* h, const uint16_t* X, int64_t n, hipStream_t s)
{
    const int N = static_cast<int>(n);
    float* g = h->grad;
    // last layer: gw3 = H2^T ds, gb3 = sum ds, dZ2 = BF16(ds w3^T * gelu'(Z2))
    colsum(h->H2, h->ds, n, h->h2, h->part, g + h->off_w3(), s);
    colsum(nullptr, h->ds, n, 1, h->part, g + h->off_b3(), s);
    hipLaunchKernelGGL(qst::k_last_bwd_dz, dim3(blocks_for(n * h->h2, 256)), dim3(256), 0, s, h->ds,
                       h->theta + h->off_w3(), h->Z2, n, h->h2, h->dZ2);
    // layer 2: gb2 = colsum dZ2, gW2 = dZ2^T H1, dZ1 = BF16((dZ2 W2) * gelu'(Z1))
    colsum(h->dZ2, nullptr, n, h->h2, h->part, g + h->off_b2(), s);
    hipLaunchKernelGGL(qst::k_transpose_bf16, dim3(blocks_for(h->h2, 32), blocks_for(n, 32)), dim3(256), 0, s, h->dZ2, N,
                       h->h2, h->dZ2T);
    hipLaunchKernelGGL(qst::k_transpose_bf16, dim3(blocks_for(h->h1, 32), blocks_for(n, 32)), dim3(256), 0, s, h->H1, N,
                       h->h1, h->H1T);
    gemm<qst::kStoreF32>(h->h2, h->h1, N, h->dZ2T, N, h->H1T, N, g + h->off_W2(), h->h1, nullptr, nullptr, nullptr,
                         nullptr, 0, s);
    hipLaunchKernelGGL(qst::k_transpose_bf16, dim3(blocks_for(h->h1, 32), blocks_for(h->h2, 32)), dim3(256), 0, s, h->W2b,
                       h->h2, h->h1, h->W2T);
    gemm<qst::kGeluGrad>(N, h->h1, h->h2, h->dZ2, h->h2, h->W2T, h->h2, nullptr, h->h1, nullptr, h->Z1, nullptr, h->dZ1,
                         h->h1, s);
    // layer 1: gb1 = colsum dZ1, gW1 = dZ1^T X
    colsum(h->dZ1, nullptr, n, h->h1, h->part, g + h->off_b1(), s);
    hipLaunchKernelGGL(qst::k_transpose_bf16, dim3(blocks_for(h->h1, 32), blocks_for(n, 32)), dim3(256), 0, s, h->dZ1, N,
                       h->h1, h->dZ1T);
    hipLaunchKernelGGL(qst::k_transpose_bf16, dim3(blocks_for(h->d, 32), blocks_for(n, 32)), dim3(256), 0, s, X, N, h->d,
                       h->XT);
    gemm<qst::kStoreF32>(h->h1, h->d, N, h->dZ1T, N, h->XT, N, g + h->off_W1(), h->d, nullptr, nullptr, nullptr, nullptr,
                         0, s);
    hipLaunchKernelGGL(qst::k_sum_f32, dim3(1), dim3(256), 0, s, h->sq, n, h->loss);
    hip_check(hipGetLastError(), "MLP backward launch");
}

void check_mlp_batch(const qst_mlp* h, int64_t n)
{
    if (!h) fail(QST_ERR_INVALID, "NULL MLP handle");
    if (n < 1) fail(QST_ERR_INVALID, "empty batch");
    if (n % 32 != 0) fail(QST_ERR_INVALID, "training batch must be a multiple of 32 rows");
    if (n > (1 << 24)) fail(QST_ERR_INVALID, "batch too large");
}

// x: [n, d] BF16 rows, y: [n] FP32 targets (y may be NULL where none is read)
void check_mlp_inputs(const qst_mlp* h, const uint16_t* x, const float* y, int64_t n, bool need_y = true)
{
    if (!x || (need_y && !y)) fail(QST_ERR_INVALID, "NULL batch");
    check_device_buffer(x, static_cast<size_t>(n) * h->d * sizeof(uint16_t), h->device, "x");
    if (y) check_device_buffer(y, static_cast<size_t>(n) * sizeof(float), h->device, "y");
}

}  // namespace

extern "C" {

qst_status qst_mlp_create(int32_t d_in, int32_t h1, int32_t h2, int32_t device, qst_mlp** out)
{
    return guarded([&] {
        if (!out) fail(QST_ERR_INVALID, "NULL output");
        *out = nullptr;
        if (d_in < 32 || d_in % 32 != 0) fail(QST_ERR_INVALID, "input width must be a positive multiple of 32");
        if (h1 < 32 || h1 % 32 != 0 || h2 < 32 || h2 % 32 != 0 || h1 > 8192 || h2 > 8192)
            fail(QST_ERR_INVALID, "hidden widths must be multiples of 32 in 32..8192");
        int ndev = 0;
        hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (device < 0 || device >= ndev) fail(QST_ERR_INVALID, "bad device ordinal");
        DeviceGuard g(device);
        auto h = std::make_unique<qst_mlp>();
        h->d = d_in;
        h->h1 = h1;
        h->h2 = h2;
        h->device = device;
        h->n_par = h->off_b3() + 1;
        try {
            h->theta = dev_alloc<float>(h->n_par);
            h->grad = dev_alloc<float>(h->n_par);
            h->m = dev_alloc<float>(h->n_par);
            h->v = dev_alloc<float>(h->n_par);
            h->W1b = dev_alloc<uint16_t>(static_cast<size_t>(h1) * d_in);
            h->W2b = dev_alloc<uint16_t>(static_cast<size_t>(h2) * h1);
            h->W2T = dev_alloc<uint16_t>(static_cast<size_t>(h2) * h1);
            for (float* p : {h->theta, h->grad, h->m, h->v})
                hip_check(hipMemset(p, 0, sizeof(float) * h->n_par), "zero MLP state");
            mlp_refresh_bf16(h.get(), nullptr);
            hip_check(hipDeviceSynchronize(), "MLP init");
        } catch (...) {
            h->free_all();
            throw;
        }
        *out = h.release();
    });
}

void qst_mlp_free(qst_mlp* h)
{
    if (!h) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    h->free_all();
    (void)hipSetDevice(prev);
    delete h;
}

int64_t qst_mlp_num_params(const qst_mlp* h) { return h ? h->n_par : -1; }

qst_status qst_mlp_set_params(qst_mlp* h, const float* params, int64_t n, float out_scale, float out_shift)
{
    return guarded([&] {
        if (!h || !params) fail(QST_ERR_INVALID, "NULL argument");
        if (n != h->n_par) fail(QST_ERR_INVALID, "parameter count mismatch");
        DeviceGuard g(h->device);
        hip_check(hipMemcpy(h->theta, params, sizeof(float) * n, hipMemcpyHostToDevice), "copy parameters");
        for (float* p : {h->m, h->v}) hip_check(hipMemset(p, 0, sizeof(float) * h->n_par), "reset Adam");
        h->t = 0;
        h->out_scale = out_scale;
        h->out_shift = out_shift;
        mlp_refresh_bf16(h, nullptr);
        hip_check(hipDeviceSynchronize(), "set parameters");
    });
}

qst_status qst_mlp_get_params(const qst_mlp* h, float* params, int64_t n)
{
    return guarded([&] {
        if (!h || !params) fail(QST_ERR_INVALID, "NULL argument");
        if (n != h->n_par) fail(QST_ERR_INVALID, "parameter count mismatch");
        DeviceGuard g(h->device);
        hip_check(hipDeviceSynchronize(), "sync");
        hip_check(hipMemcpy(params, h->theta, sizeof(float) * n, hipMemcpyDeviceToHost), "copy parameters");
    });
}

qst_status qst_mlp_gradients(qst_mlp* h, const uint16_t* x, const float* y, int64_t n, float* grad_host,
                             float* loss_host, void* stream)
{
    return guarded([&] {
        check_mlp_batch(h, n);
        check_mlp_inputs(h, x, y, n);
        DeviceGuard g(h->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        mlp_forward(h, x, n, nullptr, y, s);
        mlp_backward(h, x, n, s);
        hip_check(hipStreamSynchronize(s), "gradients synchronize");
        if (grad_host)
            hip_check(hipMemcpy(grad_host, h->grad, sizeof(float) * h->n_par, hipMemcpyDeviceToHost), "copy gradients");
        if (loss_host) {
            float l = 0.0f;
            hip_check(hipMemcpy(&l, h->loss, sizeof(float), hipMemcpyDeviceToHost), "copy loss");
            *loss_host = l / static_cast<float>(n);
        }
    });
}

qst_status qst_mlp_train_step(qst_mlp* h, const uint16_t* x, const float* y, int64_t n, float lr, float* loss_host,
                              void* stream)
{
    return guarded([&] {
        check_mlp_batch(h, n);
        check_mlp_inputs(h, x, y, n);
        if (!(lr > 0.0f)) fail(QST_ERR_INVALID, "learning rate must be positive");
        DeviceGuard g(h->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        mlp_forward(h, x, n, nullptr, y, s);
        mlp_backward(h, x, n, s);
        h->t += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float bc1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(h->t)));
        const float bc2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(h->t)));
        hipLaunchKernelGGL(qst::k_adam, dim3(blocks_for(h->n_par, 256)), dim3(256), 0, s, h->theta, h->grad, h->m, h->v,
                           h->n_par, lr, 0.9f, 0.999f, 1e-8f, bc1, bc2);
        hip_check(hipGetLastError(), "Adam launch");
        mlp_refresh_bf16(h, s);
        if (loss_host) {
            hip_check(hipStreamSynchronize(s), "train synchronize");
            float l = 0.0f;
            hip_check(hipMemcpy(&l, h->loss, sizeof(float), hipMemcpyDeviceToHost), "copy loss");
            *loss_host = l / static_cast<float>(n);
        }
    });
}

qst_status qst_mlp_predict(qst_mlp* h, const uint16_t* x, int64_t n, float* out, void* stream)
{
    return guarded([&] {
        if (!h || !x || !out) fail(QST_ERR_INVALID, "NULL argument");
        if (n < 1) fail(QST_ERR_INVALID, "empty batch");
        check_mlp_inputs(h, x, nullptr, n, false);
        check_device_buffer(out, static_cast<size_t>(n) * sizeof(float), h->device, "out");
        DeviceGuard g(h->device);
        mlp_forward(h, x, n, out, nullptr, static_cast<hipStream_t>(stream));
    });
}

qst_status qst_mlp_targets(const double* ll, int64_t n, float* y, double* mean, double* sd, void* stream)
{
    return guarded([&] {
        if (!ll || !y || !mean || !sd) fail(QST_ERR_INVALID, "NULL argument");
        if (n < 2) fail(QST_ERR_INVALID, "need at least two targets");
        const int dev = current_device();
        check_device_buffer(ll, static_cast<size_t>(n) * sizeof(double), dev, "ll");
        check_device_buffer(y, static_cast<size_t>(n) * sizeof(float), dev, "y");
        hipStream_t s = static_cast<hipStream_t>(stream);
        double* mom = dev_alloc<double>(3);
        double host[3] = {0.0, 0.0, 0.0};
        try {
            hipLaunchKernelGGL(qst::k_moments_f64, dim3(1), dim3(256), 0, s, ll, n, mom);
            hip_check(hipGetLastError(), "target moments");
            hip_check(hipStreamSynchronize(s), "target moments");
            hip_check(hipMemcpy(host, mom, sizeof(host), hipMemcpyDeviceToHost), "target moments");
        } catch (...) {
            dev_free(mom);
            throw;
        }
        dev_free(mom);
        if (host[2] != 0.0) fail(QST_ERR_INVALID, "non-finite training target");
        const double sdv = std::sqrt(host[1]);
        if (!(sdv > 0.0)) fail(QST_ERR_INVALID, "constant training targets");
        hipLaunchKernelGGL(qst::k_standardise, dim3(blocks_for(n, 256)), dim3(256), 0, s, ll, n, host[0], sdv, y);
        hip_check(hipGetLastError(), "standardise");
        *mean = host[0];
        *sd = sdv;
    });
}

qst_status qst_gather_rows(const uint16_t* x, int32_t width, const float* y, int64_t n_rows, const int64_t* idx,
                           int64_t n, uint16_t* xo, float* yo, void* stream)
{
    return guarded([&] {
        if (!x || !y || !idx || !xo || !yo) fail(QST_ERR_INVALID, "NULL argument");
        if (n < 0 || width < 1 || n_rows < 1) fail(QST_ERR_INVALID, "bad sizes");
        if (n == 0) return;
        if (n > 0x7fffffff) fail(QST_ERR_INVALID, "too many rows");
        const int dev = current_device();
        check_device_buffer(x, static_cast<size_t>(n_rows) * width * sizeof(uint16_t), dev, "x");
        check_device_buffer(y, static_cast<size_t>(n_rows) * sizeof(float), dev, "y");
        check_device_buffer(idx, static_cast<size_t>(n) * sizeof(int64_t), dev, "idx");
        check_device_buffer(xo, static_cast<size_t>(n) * width * sizeof(uint16_t), dev, "xo");
        check_device_buffer(yo, static_cast<size_t>(n) * sizeof(float), dev, "yo");
        // every index must name a row of x and y: checked on the host before
        // the gather is queued, after the work already on the stream (which
        // may be writing idx)
        const hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<int64_t> host(static_cast<size_t>(n));
        hip_check(hipStreamSynchronize(s), "gather synchronize");
        hip_check(hipMemcpy(host.data(), idx, sizeof(int64_t) * host.size(), hipMemcpyDeviceToHost), "idx copy");
        for (int64_t k = 0; k < n; ++k)
            if (host[k] < 0 || host[k] >= n_rows)
                fail(QST_ERR_INVALID, "idx[" + std::to_string(k) + "] = " + std::to_string(host[k]) +
                                          " is not a row index in [0, " + std::to_string(n_rows) + ")");
        hipLaunchKernelGGL(qst::k_gather_rows, dim3(static_cast<unsigned>(n)), dim3(256), 0, s, x, width, y, idx, n,
                           xo, yo);
        hip_check(hipGetLastError(), "gather launch");
    });
}

qst_status qst_mlp_surrogate(const qst_mlp* h, qst_surrogate* out)
{
    return guarded([&] {
        if (!h || !out) fail(QST_ERR_INVALID, "NULL argument");
        out->h1 = h->h1;
        out->h2 = h->h2;
        out->W1 = h->W1b;
        out->b1 = h->theta + h->off_b1();
        out->W2 = h->W2b;
        out->b2 = h->theta + h->off_b2();
        out->w3 = h->theta + h->off_w3();
        out->b3 = 0.0f;   // read from the device copy by the delayed-acceptance path
        out->out_scale = h->out_scale;
        out->out_shift = h->out_shift;
        out->model = const_cast<qst_mlp*>(h);
    });
}

}  // extern "C"

// ===========================================================================
// Delayed acceptance: the per-step launch sequence
// ===========================================================================
namespace {

// Team shape of the delayed-acceptance kernels per qubit count (the tuned
// single-problem defaults).
Shape da_shape(int Q) { return Shape{Q == 1 ? 8 : Q == 2 ? 16 : Q == 3 ? 32 : Q == 4 ? 64 : Q == 5 ? 256 : 512,
                                     Q <= 3 ? 64 : Q == 4 ? 256 : Q == 5 ? 256 : 512}; }

template <typename T>
void fill_zero(T* p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL((qst::k_fill_zero<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
    hip_check(hipGetLastError(), "clear");
}

template <int Q, int G, int WG>
void da_steps(qst_problem* p, const qst_run_desc& r, qst_mlp* net, qst::DaArgs P, hipStream_t s)
{
    using Dm = qst::Dims<Q>;
    using S = qst::TeamShape<Q, G>;
    const int64_t teams = WG / G;
    const unsigned blocks = static_cast<unsigned>((p->R + teams - 1) / teams);
    const size_t lds_prop = (2 * qst::kLogTableSize + static_cast<size_t>(teams) * (Dm::d + 4)) * sizeof(double);
    const size_t lds_exact = (static_cast<size_t>(teams) * S::kLds + qst::WgTables<Q>::kDoubles) * sizeof(double);
    allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_da_propose<Q, G, WG>), lds_prop);
    allow_dynamic_lds(reinterpret_cast<const void*>(&qst::k_da_exact<Q, G, WG>), lds_exact);
    for (int64_t t = 0; t < r.n_steps; ++t) {
        P.j = p->step + 1 + t;
        P.t = t;
        hipLaunchKernelGGL((qst::k_da_propose<Q, G, WG>), dim3(blocks), dim3(WG), lds_prop, s, P);
        mlp_forward(net, p->xb, p->R, p->smlp, nullptr, s);
        hipLaunchKernelGGL(qst::k_zero_counter, dim3(1), dim3(1), 0, s, p->n_surv);
        hipLaunchKernelGGL((qst::k_da_stage1<Q>), dim3(static_cast<unsigned>((p->R + 3) / 4)), dim3(256), 0, s, P);
        hipLaunchKernelGGL((qst::k_da_exact<Q, G, WG>), dim3(blocks), dim3(WG), lds_exact, s, P);
        hip_check(hipGetLastError(), "delayed-acceptance step launch");
    }
}

void launch_da(qst_problem* p, const qst_run_desc& r, hipStream_t s)
{
    qst_mlp* net = r.surrogate->model;
    if (net->device != p->device) fail(QST_ERR_INVALID, "surrogate lives on another device");
    if (net->d != p->da_width())
        fail(QST_ERR_INVALID, "surrogate input width must be 2D^2+D rounded up to a multiple of 32");
    p->ensure_da();
    const Shape sh = da_shape(p->Q);
    // step 0 (or the resumed state) by the plain kernel, then s(y) of the current states
    if (!r.resume) {
        qst_run_desc r0 = r;
        r0.n_steps = 0;
        r0.surrogate = nullptr;
        qst::ChainArgs a0 = make_args(p, r0);
        launch_chains(p->Q, sh, qst::kPathKron, qst::kPrecF64, a0, p->chain0, s);
    }
    const int dp = p->da_width();
    hipLaunchKernelGGL(qst::k_rows_to_bf16, dim3(blocks_for(p->R * dp, 256)), dim3(256), 0, s, p->x, p->R, p->d, dp,
                       p->xb);
    mlp_forward(net, p->xb, p->R, p->smlp, nullptr, s);
    hipLaunchKernelGGL(qst::k_f32_to_f64, dim3(blocks_for(p->R, 256)), dim3(256), 0, s, p->smlp, p->R, p->s_cur);
    fill_zero(p->n_stage1, p->R, s);
    fill_zero(p->nacc, p->R, s);
    fill_zero(p->nnear, p->R, s);
    hip_check(hipGetLastError(), "delayed-acceptance setup");
    qst::DaArgs P{};
    P.A = make_args(p, r, false);   // local chain indices; the propose kernel adds chain0
    P.chain0 = p->chain0;
    P.s_cur = p->s_cur;
    P.n_stage1 = p->n_stage1;
    P.yprop = p->yprop;
    P.xb = p->xb;
    P.dp = dp;
    P.smlp = p->smlp;
    P.u_mh = p->u_mh;
    P.u_da = p->u_da;
    P.surv = p->surv;
    P.n_surv = p->n_surv;
    switch (p->Q) {
        case 1: return da_steps<1, 8, 64>(p, r, net, P, s);
        case 2: return da_steps<2, 16, 64>(p, r, net, P, s);
        case 3: return da_steps<3, 32, 64>(p, r, net, P, s);
        case 4: return da_steps<4, 64, 256>(p, r, net, P, s);
        case 5: return da_steps<5, 256, 256>(p, r, net, P, s);
        default: return da_steps<6, 512, 512>(p, r, net, P, s);
    }
}

}  // namespace
