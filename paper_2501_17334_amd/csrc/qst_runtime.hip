// Host runtime and C ABI of the gfx950 pooled-pCN tomography library.
//
// Owns every device buffer behind a qst_problem handle, validates arguments,
// picks a launch shape per qubit count, and turns each call of the ABI into
// kernel launches on the caller's stream.  See include/qst.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qst.h"
#include "acf_kernel.hpp"
#include "chain_kernel.hpp"
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

// Launch shape of the chain kernel for one qubit count: team size G (threads
// per chain) and workgroup size WG.
struct Shape {
    int G, WG;
};

Shape default_shape(int Q)
{
    switch (Q) {
        case 1: return {8, 64};
        case 2: return {16, 64};
        case 3: return {32, 64};
        case 4: return {64, 64};
        case 5: return {64, 64};
        default: return {256, 256};
    }
}

template <int Q, int G, int WG>
void launch_chains_t(const qst::ChainArgs& a, hipStream_t s)
{
    using S = qst::TeamShape<Q, G>;
    const int64_t teams = WG / G;
    const int64_t blocks = (a.R + teams - 1) / teams;
    const size_t lds = (static_cast<size_t>(teams) * S::kLds + qst::WgTables<Q>::kDoubles) * sizeof(double);
    static bool attr_done = false;
    if (!attr_done) {
        hip_check(hipFuncSetAttribute(reinterpret_cast<const void*>(&qst::k_chains<Q, G, WG>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)),
                  "hipFuncSetAttribute");
        attr_done = true;
    }
    if (blocks > 0x7fffffff) fail(QST_ERR_INVALID, "too many chains for one launch");
    hipLaunchKernelGGL((qst::k_chains<Q, G, WG>), dim3(static_cast<unsigned>(blocks)), dim3(WG), lds, s, a);
    hip_check(hipGetLastError(), "chain kernel launch");
}

template <int Q, int G, int WG>
void launch_loglik_t(const double* nd, const double* rho, int64_t n, double* out, hipStream_t s)
{
    using S = qst::TeamShape<Q, G>;
    const int64_t teams = WG / G;
    const int64_t blocks = (n + teams - 1) / teams;
    const size_t lds = (static_cast<size_t>(teams) * S::kLds + qst::WgTables<Q>::kDoubles) * sizeof(double);
    static bool attr_done = false;
    if (!attr_done) {
        hip_check(hipFuncSetAttribute(reinterpret_cast<const void*>(&qst::k_loglik<Q, G, WG>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)),
                  "hipFuncSetAttribute");
        attr_done = true;
    }
    hipLaunchKernelGGL((qst::k_loglik<Q, G, WG>), dim3(static_cast<unsigned>(blocks)), dim3(WG), lds, s, nd,
                       rho, n, out);
    hip_check(hipGetLastError(), "loglik kernel launch");
}

void launch_chains(int Q, Shape sh, const qst::ChainArgs& a, hipStream_t s)
{
#define QST_CASE(q, g, wg) \
    if (Q == q && sh.G == g && sh.WG == wg) return launch_chains_t<q, g, wg>(a, s);
    QST_CASE(1, 8, 64)
    QST_CASE(2, 16, 64)
    QST_CASE(3, 32, 64)
    QST_CASE(4, 64, 64)
    QST_CASE(5, 64, 64)
    QST_CASE(6, 256, 256)
#undef QST_CASE
    fail(QST_ERR_UNSUPPORTED, "no chain kernel for Q=" + std::to_string(Q) + " G=" + std::to_string(sh.G));
}

void launch_loglik(int Q, const double* nd, const double* rho, int64_t n, double* out, hipStream_t s)
{
    switch (Q) {
        case 1: return launch_loglik_t<1, 8, 64>(nd, rho, n, out, s);
        case 2: return launch_loglik_t<2, 16, 64>(nd, rho, n, out, s);
        case 3: return launch_loglik_t<3, 32, 64>(nd, rho, n, out, s);
        case 4: return launch_loglik_t<4, 64, 64>(nd, rho, n, out, s);
        case 5: return launch_loglik_t<5, 64, 64>(nd, rho, n, out, s);
        case 6: return launch_loglik_t<6, 256, 256>(nd, rho, n, out, s);
    }
    fail(QST_ERR_INVALID, "bad Q");
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
    std::vector<int64_t> counts;
    double* nd = nullptr;  // counts as doubles
    // chain state
    int64_t R = 0;
    int64_t step = 0;
    bool have_run = false;
    double *x = nullptr, *ll = nullptr, *beta = nullptr, *rho = nullptr, *s1 = nullptr, *s2 = nullptr;
    int32_t* accw = nullptr;
    int64_t *nst = nullptr, *nacc = nullptr, *nnear = nullptr;
    hipStream_t last_stream = nullptr;

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
    if (r.resume) {
        if (!p->have_run) fail(QST_ERR_STATE, "resume requested before any run of this handle");
        if (r.n_chains != p->R) fail(QST_ERR_INVALID, "resume with a different n_chains");
    }
    if (r.surrogate) fail(QST_ERR_UNSUPPORTED, "delayed acceptance is not available in this build");
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
        p->d = 2 * p->D2 + p->D;
        p->K = ipow3(Q);
        p->KD = p->K * p->D;
        p->device = desc->device;
        p->precision = desc->precision;
        p->path = desc->path == QST_PATH_AUTO ? QST_PATH_KRON : desc->path;
        if (p->path == QST_PATH_DENSE || p->precision != QST_FP64)
            fail(QST_ERR_UNSUPPORTED, "only the FP64 Kronecker path is available in this build");
        p->counts.assign(desc->counts, desc->counts + p->KD);
        std::vector<double> nd(p->KD);
        for (int i = 0; i < p->KD; ++i) {
            if (p->counts[i] < 0) fail(QST_ERR_INVALID, "negative count");
            nd[i] = static_cast<double>(p->counts[i]);
        }
        DeviceGuard g(p->device);
        p->nd = dev_alloc<double>(p->KD);
        hip_check(hipMemcpy(p->nd, nd.data(), sizeof(double) * p->KD, hipMemcpyHostToDevice), "copy counts");
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
    (void)hipSetDevice(prev);
    delete p;
}

qst_status qst_run_chains(qst_problem* const* problems, int32_t n_problems, const qst_run_desc* runs,
                          qst_run_stats* stats)
{
    return guarded([&] {
        if (!problems || !runs || n_problems < 1) fail(QST_ERR_INVALID, "empty batch");
        const int dev = problems[0] ? problems[0]->device : 0;
        for (int i = 0; i < n_problems; ++i) {
            if (!problems[i]) fail(QST_ERR_INVALID, "NULL problem handle");
            if (problems[i]->device != dev) fail(QST_ERR_INVALID, "batch spans several devices");
            validate_run(problems[i], runs[i]);
        }
        if (n_problems > 1) fail(QST_ERR_UNSUPPORTED, "batched launch is not available in this build");
        DeviceGuard g(dev);
        qst_problem* p = problems[0];
        const qst_run_desc& r = runs[0];
        hipStream_t s = static_cast<hipStream_t>(r.stream);
        if (!r.resume) {
            if (p->R != r.n_chains) {
                if (p->last_stream) hip_check(hipStreamSynchronize(p->last_stream), "sync before realloc");
                p->alloc_state(r.n_chains);
            }
            p->step = 0;
        }
        qst::ChainArgs a{};
        a.nd = p->nd;
        a.R = p->R;
        a.x = p->x;
        a.ll = p->ll;
        a.beta = p->beta;
        a.acc_win = p->accw;
        a.rho_cur = p->rho;
        a.s1 = p->s1;
        a.s2 = p->s2;
        a.n_stored = p->nst;
        a.n_acc = p->nacc;
        a.n_near = p->nnear;
        a.step_begin = p->step;
        a.n_steps = r.n_steps;
        a.burn_in = r.burn_in;
        a.adapt_until = r.adapt_until;
        a.thin = r.thin;
        a.adapt_every = r.adapt_every;
        a.init = r.resume ? 0 : 1;
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
        launch_chains(p->Q, default_shape(p->Q), a, s);
        p->step += r.n_steps;
        p->have_run = true;
        p->last_stream = s;
        if (stats) {
            hip_check(hipStreamSynchronize(s), "run synchronize");
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
            stats[0] = st;
        }
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
            hipLaunchKernelGGL(qst::k_pool_final, dim3(1), dim3(qst::kPoolThreads), 0, s, part, nsum, nchunks, p->D,
                               outd, nout);
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

qst_status qst_loglik(const qst_problem* p, const double* rho, int64_t n, double* ll_out, qst_path path,
                      qst_precision precision, void* stream)
{
    return guarded([&] {
        if (!p) fail(QST_ERR_INVALID, "NULL handle");
        if (n < 0) fail(QST_ERR_INVALID, "negative n");
        if (n == 0) return;
        if (!rho || !ll_out) fail(QST_ERR_INVALID, "NULL buffer");
        const qst_path pth = path == QST_PATH_AUTO ? p->path : path;
        if (pth != QST_PATH_KRON || precision != QST_FP64)
            fail(QST_ERR_UNSUPPORTED, "only the FP64 Kronecker path is available in this build");
        DeviceGuard g(p->device);
        launch_loglik(p->Q, p->nd, rho, n, ll_out, static_cast<hipStream_t>(stream));
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
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int D = 1 << n_qubits;
        double* part = dev_alloc<double>(static_cast<size_t>(n_chains) * (l_max + 1));
        double* outd = nullptr;
        try {
            outd = dev_alloc<double>(l_max + 1);
            const dim3 grid((l_max + 1 + qst::kAcfLags - 1) / qst::kAcfLags, static_cast<unsigned>(n_chains));
            hipLaunchKernelGGL(qst::k_acf_partial, grid, dim3(qst::kAcfThreads), 0, s, records, n_samples, D, l_max,
                               part);
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
