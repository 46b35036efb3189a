// sv_api.cpp -- host runtime behind the C ABI of include/sv.h: state
// handles, argument validation, gate classification and kernel dispatch,
// expectation values and the adjoint driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "sv_internal.h"

namespace sv {

namespace {
thread_local std::string g_last_error;
// the state the current entry point validated (check_state); a HIP failure
// during the call marks it failed
thread_local sv_state g_active = nullptr;
}

[[noreturn]] void fail(sv_status st, const std::string& msg) { throw Error{st, msg}; }

void set_last_error(const std::string& msg) { g_last_error = msg; }

void gate_matrix_of_op(const sv_op& op, const double* params, cd* m, int* k)
{
    if (op.kind == SV_MATRIX) {
        if (!op.matrix) fail(SV_ERR_INVALID_ARGUMENT, "SV_MATRIX op without a matrix");
        *k = op.n_targets;
        const int D = 1 << *k;
        for (int i = 0; i < D * D; ++i) m[i] = cd(op.matrix[2 * i], op.matrix[2 * i + 1]);
        return;
    }
    double prm[3] = {0.0, 0.0, 0.0};
    const int np = kind_nparams(op.kind);
    for (int j = 0; j < np; ++j) prm[j] = params[op.param[j]];
    *k = kind_matrix(op.kind, prm, m);
    if (*k < 0) fail(SV_ERR_INVALID_ARGUMENT, "unknown gate kind " + std::to_string(op.kind));
}

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) fail(SV_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

const DeviceInfo& device_info()
{
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = 0;
    SV_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        DeviceInfo d;
        d.device = dev;
        SV_HIP(hipDeviceGetAttribute(&d.cu_count, hipDeviceAttributeMultiprocessorCount, dev));
        it = cache.emplace(dev, d).first;
    }
    return it->second;
}

namespace {

template <class F>
sv_status guarded(F&& f)
{
    g_active = nullptr;
    try {
        f();
        g_last_error.clear();
        g_active = nullptr;
        return SV_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        if (e.st == SV_ERR_HIP && g_active && !g_active->failed) {
            // sticky: the state's contents are undefined from here on
            g_active->failed = true;
            g_active->failed_msg = e.msg;
        }
        g_active = nullptr;
        return e.st;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return SV_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SV_ERR_INVALID_ARGUMENT;
    } catch (...) {
        g_last_error = "unknown error";
        return SV_ERR_INVALID_ARGUMENT;
    }
}

void need(bool ok, sv_status st, const std::string& msg)
{
    if (!ok) fail(st, msg);
}

// ------------------------------------------------------------ validation

void check_gate(int n, const int* targets, int nt, const int* controls, int nc, int max_k)
{
    need(nt >= 1 && nt <= max_k, SV_ERR_UNSUPPORTED, "number of targets must be 1.." + std::to_string(max_k));
    need(nc >= 0 && nc <= SV_MAX_CONTROLS, SV_ERR_UNSUPPORTED, "at most 3 controls");
    need(targets != nullptr, SV_ERR_INVALID_ARGUMENT, "targets is NULL");
    need(nc == 0 || controls != nullptr, SV_ERR_INVALID_ARGUMENT, "controls is NULL");
    need(nt + nc <= n, SV_ERR_UNSUPPORTED, "more gate qubits than state qubits");
    uint64_t seen = 0;
    auto one = [&](int q) {
        need(q >= 0 && q < n, SV_ERR_QUBIT_OUT_OF_RANGE,
             "qubit " + std::to_string(q) + " out of range for n=" + std::to_string(n));
        need(!((seen >> q) & 1), SV_ERR_QUBIT_OVERLAP, "qubit " + std::to_string(q) + " used twice");
        seen |= 1ull << q;
    };
    for (int j = 0; j < nt; ++j) one(targets[j]);
    for (int j = 0; j < nc; ++j) one(controls[j]);
}

void check_state(sv_state s)
{
    need(s != nullptr && s->psi != nullptr, SV_ERR_INVALID_ARGUMENT, "null state");
    need(!s->failed, SV_ERR_HIP, "the state is unusable after an earlier HIP error (" + s->failed_msg + ")");
    g_active = s;
    if (s->inject_hip_error) {
        s->inject_hip_error = false;
        fail(SV_ERR_HIP, "injected HIP error (testing hook)");
    }
}

void check_not_capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SV_HIP(hipStreamIsCapturing(st, &cs));
    need(cs == hipStreamCaptureStatusNone, SV_ERR_CAPTURE, "synchronising call on a capturing stream");
}

// ------------------------------------------------------------ scratch

void ensure_scratch(sv_state s, uint64_t doubles)
{
    if (doubles <= s->scratch_cap) return;
    if (s->scratch) {
        SV_HIP(hipStreamSynchronize(s->stream));
        SV_HIP(hipFree(s->scratch));
        s->scratch = nullptr;
        s->scratch_cap = 0;
    }
    if (hipMalloc(&s->scratch, doubles * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        s->scratch = nullptr;
        fail(SV_ERR_OUT_OF_MEMORY, "reduction scratch allocation failed");
    }
    s->scratch_cap = doubles;
}

void ensure_dout(sv_state s, uint64_t doubles)
{
    if (doubles <= s->dout_cap) return;
    if (s->dout) {
        SV_HIP(hipStreamSynchronize(s->stream));
        SV_HIP(hipFree(s->dout));
        SV_HIP(hipHostFree(s->hout));
        s->dout = nullptr;
        s->hout = nullptr;
        s->dout_cap = 0;
    }
    const uint64_t cap = std::max<uint64_t>(doubles, 1024);
    if (hipMalloc(&s->dout, cap * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        fail(SV_ERR_OUT_OF_MEMORY, "output buffer allocation failed");
    }
    SV_HIP(hipHostMalloc(&s->hout, cap * sizeof(double), hipHostMallocDefault));
    s->dout_cap = cap;
}

void ensure_hstage(sv_state s, uint64_t floats)
{
    if (floats <= s->hstage_cap) return;
    if (s->hstage) {
        SV_HIP(hipStreamSynchronize(s->stream));
        SV_HIP(hipHostFree(s->hstage));
        s->hstage = nullptr;
        s->hstage_cap = 0;
    }
    const uint64_t cap = std::max<uint64_t>(floats, 4096);
    SV_HIP(hipHostMalloc(&s->hstage, cap * sizeof(float), hipHostMallocDefault));
    s->hstage_cap = cap;
}

constexpr int kAmEvents = 16;
static_assert(sizeof(sv_state_s::events) / sizeof(hipEvent_t) == kAmEvents, "one event per chunk");

void ensure_events(sv_state s)
{
    for (int i = 0; i < kAmEvents; ++i)
        if (!s->events[i]) SV_HIP(hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming));
}

// copy `doubles` results from dout to hout and wait
void fetch(sv_state s, uint64_t doubles)
{
    SV_HIP(hipMemcpyAsync(s->hout, s->dout, doubles * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
}

Rows all_rows(sv_state s) { return Rows{s->psi, s->psi, s->batch, s->batch, s->N}; }
Rows one_row(sv_state s, float2* base, int r) { return Rows{base + (uint64_t)r * s->N, base, 1, 1, s->N}; }

// ------------------------------------------------------------ gate dispatch

bool is_exact(cd v, double re) { return v.real() == re && v.imag() == 0.0; }

float2 f2(cd v) { return make_float2((float)v.real(), (float)v.imag()); }

// Apply (M, targets, controls) to the given rows, choosing the kernel by the
// matrix structure: diagonal -> phase sweep (only the changed subspace when
// M differs from I in its last entry alone), otherwise dense group update.
void dispatch(const Rows& rows, int k, const int* targets, int nc, const int* controls, const cd* m,
              hipStream_t st)
{
    const int D = 1 << k;
    bool diag = true, ident = true, ones = true;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            const cd v = m[r * D + c];
            if (r != c && v != cd(0.0)) diag = false;
            if (!is_exact(v, r == c ? 1.0 : 0.0)) ident = false;
            if (r == c && r != D - 1 && !is_exact(v, 1.0)) ones = false;
        }
    if (ident) return;
    if (diag) {
        DiagLaunch d{};
        d.rows = rows;
        for (int j = 0; j < nc; ++j) d.fixed[d.nfixed++] = controls[j];
        if (ones) {
            for (int j = 0; j < k; ++j) d.fixed[d.nfixed++] = targets[j];
            d.nfree = 0;
            d.ph[0] = f2(m[(D - 1) * D + D - 1]);
        } else {
            d.nfree = k;
            for (int j = 0; j < k; ++j) d.freeq[j] = targets[j];
            for (int r = 0; r < D; ++r) d.ph[r] = f2(m[r * D + r]);
        }
        launch_diag(d, st);
        return;
    }
    GateLaunch g{};
    g.rows = rows;
    g.k = k;
    for (int j = 0; j < k; ++j) g.targets[j] = targets[j];
    g.nc = nc;
    for (int j = 0; j < nc; ++j) g.controls[j] = controls[j];
    for (int i = 0; i < D * D; ++i) g.m[i] = f2(m[i]);
    launch_gate(g, st);
}

void dagger(int k, const cd* m, cd* out)
{
    const int D = 1 << k;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) out[c * D + r] = std::conj(m[r * D + c]);
}

void check_unitary(int k, const cd* m)
{
    const int D = 1 << k;
    double worst = 0.0;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            cd acc = 0.0;
            for (int j = 0; j < D; ++j) acc += m[r * D + j] * std::conj(m[c * D + j]);
            worst = std::max(worst, std::abs(acc - (r == c ? cd(1.0) : cd(0.0))));
        }
    need(worst <= 1e-6, SV_ERR_NOT_UNITARY, "matrix is not unitary (max |M M^* - I| = " + std::to_string(worst) + ")");
}

// ------------------------------------------------------------ ops

struct OpInfo {
    int k;
    int np;
};

OpInfo check_op(int n, const sv_op& op, int n_params)
{
    need(op.kind >= SV_H && op.kind <= SV_MATRIX, SV_ERR_INVALID_ARGUMENT, "unknown gate kind " + std::to_string(op.kind));
    int k = kind_targets(op.kind);
    if (op.kind == SV_MATRIX) {
        need(op.matrix != nullptr, SV_ERR_INVALID_ARGUMENT, "SV_MATRIX op without a matrix");
        k = op.n_targets;
    }
    need(op.n_targets == k, SV_ERR_INVALID_ARGUMENT, "n_targets does not match the gate kind");
    check_gate(n, op.targets, op.n_targets, op.controls, op.n_controls, SV_MAX_GATE_TARGETS);
    const int np = op.kind == SV_MATRIX ? 0 : kind_nparams(op.kind);
    for (int j = 0; j < np; ++j)
        need(op.param[j] >= 0 && op.param[j] < n_params, SV_ERR_INVALID_ARGUMENT,
             "parameter index " + std::to_string(op.param[j]) + " out of range");
    return OpInfo{k, np};
}

// matrix of op for parameter row `prow`
void op_matrix(const sv_op& op, const OpInfo& info, const double* prow, cd* m)
{
    if (op.kind == SV_MATRIX) {
        const int D = 1 << info.k;
        for (int i = 0; i < D * D; ++i) m[i] = cd(op.matrix[2 * i], op.matrix[2 * i + 1]);
        return;
    }
    double prm[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < info.np; ++j) prm[j] = prow[op.param[j]];
    kind_matrix(op.kind, prm, m);
}

void op_params(const sv_op& op, const OpInfo& info, const double* prow, double* prm)
{
    prm[0] = prm[1] = prm[2] = 0.0;
    for (int j = 0; j < info.np; ++j) prm[j] = prow[op.param[j]];
}

void ensure_lambda(sv_state s, void* user, float2** lam)
{
    if (user) {
        need((reinterpret_cast<uintptr_t>(user) & 15) == 0, SV_ERR_INVALID_ARGUMENT, "lambda buffer must be 16-byte aligned");
        *lam = static_cast<float2*>(user);
        return;
    }
    if (!s->lam) {
        if (hipMalloc(&s->lam, (uint64_t)s->batch * s->N * sizeof(float2)) != hipSuccess) {
            (void)hipGetLastError();
            s->lam = nullptr;
            fail(SV_ERR_OUT_OF_MEMORY, "adjoint buffer allocation failed");
        }
    }
    *lam = s->lam;
}

// Terms (and optional per-row coefficients, [rows][n_obs] in the caller's
// term order) to device memory kept in the state.
// every term a single-qubit Z (sum_q c_q Z_q): the observable kernel's table path
bool z_only_terms(const sv_pauli_term* obs, int n_obs)
{
    for (int i = 0; i < n_obs; ++i)
        if (obs[i].x_mask != 0 || __builtin_popcountll(obs[i].z_mask) != 1) return false;
    return n_obs > 0;
}

void upload_terms(sv_state s, const sv_pauli_term* obs, int n_obs, const double* coeff_rows, int rows,
                  PauliTermDev** out, const double** dcoeff)
{
    std::vector<PauliTermDev> t(n_obs);
    for (int i = 0; i < n_obs; ++i) {
        t[i].x_mask = obs[i].x_mask;
        t[i].z_mask = obs[i].z_mask;
        t[i].coeff = obs[i].coeff;
        t[i].y_count = __builtin_popcountll(obs[i].x_mask & obs[i].z_mask);
        t[i].orig = i;
    }
    // grouped by x_mask: the gather reads each source amplitude once per group
    std::stable_sort(t.begin(), t.end(),
                     [](const PauliTermDev& a, const PauliTermDev& b) { return a.x_mask < b.x_mask; });
    const size_t tbytes = (t.size() * sizeof(PauliTermDev) + 15) & ~size_t(15);
    const size_t cbytes = coeff_rows ? (size_t)rows * n_obs * sizeof(double) : 0;
    const size_t bytes = tbytes + cbytes;
    if (bytes > s->dterms_cap) {
        if (s->dterms) {
            SV_HIP(hipStreamSynchronize(s->stream));
            SV_HIP(hipFree(s->dterms));
            s->dterms = nullptr;
            s->dterms_cap = 0;
        }
        SV_HIP(hipMalloc(&s->dterms, bytes));
        s->dterms_cap = bytes;
    }
    unsigned char* d = static_cast<unsigned char*>(s->dterms);
    SV_HIP(hipMemcpyAsync(d, t.data(), t.size() * sizeof(PauliTermDev), hipMemcpyHostToDevice, s->stream));
    if (coeff_rows) SV_HIP(hipMemcpyAsync(d + tbytes, coeff_rows, cbytes, hipMemcpyHostToDevice, s->stream));
    // the host vector dies at return: make the copies complete first
    SV_HIP(hipStreamSynchronize(s->stream));
    *out = reinterpret_cast<PauliTermDev*>(d);
    *dcoeff = coeff_rows ? reinterpret_cast<const double*>(d + tbytes) : nullptr;
}

// True when every row's parameters of this op are bitwise equal to row 0's
// (then one launch serves all rows).
bool same_params_all_rows(const sv_op& op, const OpInfo& oi, const double* params, int64_t stride, int rows)
{
    for (int r = 1; r < rows; ++r)
        for (int d = 0; d < oi.np; ++d) {
            const double a = params[op.param[d]], b = params[r * stride + op.param[d]];
            if (std::memcmp(&a, &b, sizeof(double)) != 0) return false;
        }
    return true;
}

void check_terms(int n, const sv_pauli_term* terms, int nt)
{
    need(terms != nullptr && nt >= 1, SV_ERR_INVALID_ARGUMENT, "need at least one Pauli term");
    const uint64_t lim = n >= 64 ? ~0ull : ((1ull << n) - 1);
    for (int i = 0; i < nt; ++i)
        need((terms[i].x_mask & ~lim) == 0 && (terms[i].z_mask & ~lim) == 0, SV_ERR_QUBIT_OUT_OF_RANGE,
             "Pauli mask names a qubit >= n");
}

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_alloc(int n_qubits, int batch, void* device_buffer, void* stream, sv_state* out)
{
    return guarded([&] {
        need(out != nullptr, SV_ERR_INVALID_ARGUMENT, "out is NULL");
        *out = nullptr;
        need(n_qubits >= 1 && n_qubits <= SV_MAX_QUBITS, SV_ERR_INVALID_ARGUMENT,
             "n_qubits must be in [1, 34]");
        need(batch >= 1, SV_ERR_INVALID_ARGUMENT, "batch must be >= 1");
        need(device_buffer == nullptr || (reinterpret_cast<uintptr_t>(device_buffer) & 15) == 0,
             SV_ERR_INVALID_ARGUMENT, "device buffer must be 16-byte aligned");
        auto* s = new sv_state_s;
        s->n = n_qubits;
        s->batch = batch;
        s->N = 1ull << n_qubits;
        s->stream = static_cast<hipStream_t>(stream);
        if (device_buffer) {
            s->psi = static_cast<float2*>(device_buffer);
        } else {
            if (hipMalloc(&s->psi, (uint64_t)batch * s->N * sizeof(float2)) != hipSuccess) {
                (void)hipGetLastError();
                delete s;
                fail(SV_ERR_OUT_OF_MEMORY, "state allocation failed");
            }
            s->owns = true;
        }
        (void)device_info();
        *out = s;
    });
}

sv_status sv_free(sv_state s)
{
    return guarded([&] {
        if (!s) return;
        (void)hipStreamSynchronize(s->stream);
        if (s->owns && s->psi) (void)hipFree(s->psi);
        if (s->lam) (void)hipFree(s->lam);
        if (s->scratch) (void)hipFree(s->scratch);
        if (s->dout) (void)hipFree(s->dout);
        if (s->hout) (void)hipHostFree(s->hout);
        if (s->hstage) (void)hipHostFree(s->hstage);
        for (hipEvent_t e : s->events)
            if (e) (void)hipEventDestroy(e);
        if (s->dterms) (void)hipFree(s->dterms);
        if (s->dfused) (void)hipFree(s->dfused);
        delete s;
    });
}

sv_status sv_inject_hip_error(sv_state s)
{
    return guarded([&] {
        need(s != nullptr && s->psi != nullptr, SV_ERR_INVALID_ARGUMENT, "null state");
        s->inject_hip_error = true;
    });
}

sv_status sv_state_failed(sv_state s, int* failed)
{
    return guarded([&] {
        need(s != nullptr && s->psi != nullptr, SV_ERR_INVALID_ARGUMENT, "null state");
        need(failed != nullptr, SV_ERR_INVALID_ARGUMENT, "failed is NULL");
        *failed = s->failed ? 1 : 0;
    });
}

sv_status sv_device_ptr(sv_state s, void** out)
{
    return guarded([&] {
        check_state(s);
        need(out != nullptr, SV_ERR_INVALID_ARGUMENT, "out is NULL");
        *out = s->psi;
    });
}

sv_status sv_reset(sv_state s, uint64_t idx)
{
    return guarded([&] {
        check_state(s);
        need(idx < s->N, SV_ERR_INVALID_ARGUMENT, "basis index out of range");
        launch_basis(all_rows(s), idx, s->stream);
    });
}

sv_status sv_copy_state(sv_state s, void* host, int to_host)
{
    return guarded([&] {
        check_state(s);
        need(host != nullptr, SV_ERR_INVALID_ARGUMENT, "host is NULL");
        check_not_capturing(s->stream);
        const size_t bytes = (size_t)s->batch * s->N * sizeof(float2);
        if (to_host)
            SV_HIP(hipMemcpyAsync(host, s->psi, bytes, hipMemcpyDeviceToHost, s->stream));
        else
            SV_HIP(hipMemcpyAsync(s->psi, host, bytes, hipMemcpyHostToDevice, s->stream));
        SV_HIP(hipStreamSynchronize(s->stream));
    });
}

sv_status sv_check_gate(int n_qubits, const int* targets, int n_targets, const int* controls, int n_controls)
{
    return guarded([&] {
        need(n_qubits >= 1 && n_qubits <= SV_MAX_QUBITS, SV_ERR_INVALID_ARGUMENT, "n_qubits must be in [1, 34]");
        check_gate(n_qubits, targets, n_targets, controls, n_controls, SV_MAX_GATE_TARGETS);
    });
}

sv_status sv_apply_gate(sv_state s, const int* targets, int n_targets, const int* controls, int n_controls,
                        const double* matrix, int64_t matrix_batch_stride, unsigned flags)
{
    return guarded([&] {
        check_state(s);
        check_gate(s->n, targets, n_targets, controls, n_controls, SV_MAX_GATE_TARGETS);
        need(matrix != nullptr, SV_ERR_INVALID_ARGUMENT, "matrix is NULL");
        need((flags & ~(SV_FLAG_ADJOINT | SV_FLAG_CHECK_UNITARY)) == 0, SV_ERR_INVALID_ARGUMENT, "unknown flags");
        need(matrix_batch_stride >= 0, SV_ERR_INVALID_ARGUMENT, "negative matrix stride");
        const int k = n_targets, D = 1 << k;
        const bool per_row = matrix_batch_stride != 0 && s->batch > 1;
        const int nm = per_row ? s->batch : 1;
        std::vector<cd> ms((size_t)nm * D * D);
        for (int r = 0; r < nm; ++r) {
            const double* src = matrix + 2 * r * matrix_batch_stride;
            cd* m = &ms[(size_t)r * D * D];
            for (int i = 0; i < D * D; ++i) m[i] = cd(src[2 * i], src[2 * i + 1]);
            if (flags & SV_FLAG_CHECK_UNITARY) check_unitary(k, m);
            if (flags & SV_FLAG_ADJOINT) {
                cd t[16];
                dagger(k, m, t);
                std::copy(t, t + D * D, m);
            }
        }
        if (!per_row) {
            dispatch(all_rows(s), k, targets, n_controls, controls, ms.data(), s->stream);
        } else {
            for (int r = 0; r < s->batch; ++r)
                dispatch(one_row(s, s->psi, r), k, targets, n_controls, controls, &ms[(size_t)r * D * D], s->stream);
        }
    });
}

sv_status sv_run(sv_state s, const sv_op* ops, int n_ops, const double* params, int64_t params_batch_stride,
                 int n_params)
{
    return guarded([&] {
        check_state(s);
        need(n_ops >= 0 && (n_ops == 0 || ops != nullptr), SV_ERR_INVALID_ARGUMENT, "ops is NULL");
        need(n_params >= 0 && (n_params == 0 || params != nullptr), SV_ERR_INVALID_ARGUMENT, "params is NULL");
        need(params_batch_stride >= 0, SV_ERR_INVALID_ARGUMENT, "negative params stride");
        std::vector<OpInfo> info(n_ops);
        for (int i = 0; i < n_ops; ++i) info[i] = check_op(s->n, ops[i], n_params);
        const bool per_row = params_batch_stride != 0 && s->batch > 1;
        for (int i = 0; i < n_ops; ++i) {
            const sv_op& op = ops[i];
            cd m[16];
            if (!per_row || info[i].np == 0 || same_params_all_rows(op, info[i], params, params_batch_stride, s->batch)) {
                op_matrix(op, info[i], params, m);
                dispatch(all_rows(s), info[i].k, op.targets, op.n_controls, op.controls, m, s->stream);
            } else {
                for (int r = 0; r < s->batch; ++r) {
                    op_matrix(op, info[i], params + r * params_batch_stride, m);
                    dispatch(one_row(s, s->psi, r), info[i].k, op.targets, op.n_controls, op.controls, m, s->stream);
                }
            }
        }
    });
}

sv_status sv_expval_z_all(sv_state s, double* out)
{
    return guarded([&] {
        check_state(s);
        need(out != nullptr, SV_ERR_INVALID_ARGUMENT, "out is NULL");
        check_not_capturing(s->stream);
        ensure_scratch(s, zall_parts(s->n, s->batch));
        const uint64_t nout = (uint64_t)s->batch * (s->n + 1);
        ensure_dout(s, nout);
        launch_zall(all_rows(s), s->n, s->scratch, s->dout, s->stream);
        fetch(s, nout);
        std::memcpy(out, s->hout, nout * sizeof(double));
    });
}

sv_status sv_expval_z_all_noalloc(sv_state s, double* dev_out)
{
    return guarded([&] {
        check_state(s);
        need(dev_out != nullptr, SV_ERR_INVALID_ARGUMENT, "dev_out is NULL");
        need(((uintptr_t)dev_out & 7) == 0, SV_ERR_INVALID_ARGUMENT, "dev_out must be 8-byte aligned");
        const uint64_t parts = zall_parts(s->n, s->batch);
        need(parts <= kStaticZallDoubles, SV_ERR_UNSUPPORTED,
             "batch * 2^(n - 14) * 15 partial sums (" + std::to_string(parts) +
                 ") exceed the fixed buffer of " + std::to_string(kStaticZallDoubles) + " doubles");
        launch_zall(all_rows(s), s->n, static_zall_scratch(), dev_out, s->stream);
    });
}

sv_status sv_expval_pauli(sv_state s, const sv_pauli_term* terms, int n_terms, double* out)
{
    return guarded([&] {
        check_state(s);
        need(out != nullptr, SV_ERR_INVALID_ARGUMENT, "out is NULL");
        check_terms(s->n, terms, n_terms);
        check_not_capturing(s->stream);
        // group terms by x mask, at most 8 per sweep
        std::vector<PauliGroup> groups;
        std::vector<std::vector<int>> members;
        std::map<uint64_t, std::vector<int>> byx;
        for (int t = 0; t < n_terms; ++t) byx[terms[t].x_mask].push_back(t);
        for (auto& kv : byx) {
            for (size_t i = 0; i < kv.second.size(); i += 8) {
                PauliGroup g{};
                g.x_mask = kv.first;
                std::vector<int> mem;
                for (size_t j = i; j < std::min(kv.second.size(), i + 8); ++j) {
                    const int t = kv.second[j];
                    g.z_mask[g.nt] = terms[t].z_mask;
                    g.y_count[g.nt] = __builtin_popcountll(terms[t].x_mask & terms[t].z_mask);
                    ++g.nt;
                    mem.push_back(t);
                }
                groups.push_back(g);
                members.push_back(mem);
            }
        }
        ensure_scratch(s, pauli_parts(s->n, s->batch, 8));
        ensure_dout(s, (uint64_t)s->batch * n_terms);
        uint64_t off = 0;
        std::vector<uint64_t> offs;
        for (auto& g : groups) {
            offs.push_back(off);
            launch_pauli_group(all_rows(s), s->n, g, s->scratch, s->dout + off, s->stream);
            off += (uint64_t)s->batch * g.nt;
        }
        fetch(s, off);
        for (size_t gi = 0; gi < groups.size(); ++gi)
            for (int r = 0; r < s->batch; ++r)
                for (int j = 0; j < groups[gi].nt; ++j) {
                    const int t = members[gi][j];
                    out[(size_t)r * n_terms + t] = terms[t].coeff * s->hout[offs[gi] + (uint64_t)r * groups[gi].nt + j];
                }
    });
}

}  // extern "C"

namespace {

sv_status adjoint_impl(sv_state s, const sv_op* ops, int n_ops, const double* params, int64_t params_batch_stride,
                       int n_params, const sv_pauli_term* obs, int n_obs, const double* coeff_rows,
                       void* lambda_buffer, double* grad_out, double* loss_out, double* drift_out,
                       const double* diag_w = nullptr)
{
    return guarded([&] {
        check_state(s);
        need(n_ops >= 0 && (n_ops == 0 || ops != nullptr), SV_ERR_INVALID_ARGUMENT, "ops is NULL");
        need(n_params >= 0 && (n_params == 0 || params != nullptr), SV_ERR_INVALID_ARGUMENT, "params is NULL");
        need(n_params == 0 || grad_out != nullptr, SV_ERR_INVALID_ARGUMENT, "grad_out is NULL");
        need(params_batch_stride >= 0, SV_ERR_INVALID_ARGUMENT, "negative params stride");
        if (!diag_w) check_terms(s->n, obs, n_obs);
        std::vector<OpInfo> info(n_ops);
        for (int i = 0; i < n_ops; ++i) info[i] = check_op(s->n, ops[i], n_params);
        check_not_capturing(s->stream);

        const int B = s->batch;
        const bool per_row = params_batch_stride != 0 && B > 1;
        float2* lam = nullptr;
        ensure_lambda(s, lambda_buffer, &lam);
        PauliTermDev* dterms = nullptr;
        const double* dcoeff = nullptr;
        if (!diag_w) upload_terms(s, obs, n_obs, coeff_rows, B, &dterms, &dcoeff);

        // slots: one per (parameterised op, row, derivative)
        struct Slot { int row; int param; };
        std::vector<Slot> slots;
        for (int i = 0; i < n_ops; ++i) slots.reserve(slots.size() + (size_t)B * info[i].np);
        const int G = adj_grid(s->n, 1, 0);
        uint64_t nslot_max = 0;
        for (int i = 0; i < n_ops; ++i) nslot_max += (uint64_t)B * info[i].np;
        const uint64_t red = std::max<uint64_t>(inner_parts(s->n, B), drift_parts(s->n, B));
        ensure_scratch(s, std::max<uint64_t>(nslot_max * G, 1) + red);
        double* part = s->scratch;
        double* rscratch = s->scratch + std::max<uint64_t>(nslot_max * G, 1);
        const uint64_t nout = std::max<uint64_t>(nslot_max, 1) + 3ull * B;
        ensure_dout(s, nout + 2ull * B);
        double* d_slots = s->dout;
        double* d_loss = s->dout + std::max<uint64_t>(nslot_max, 1);       // [B][2] re, im
        double* d_drift = d_loss + 2ull * B;                                // [B]

        const Rows prow{s->psi, s->psi, B, B, s->N};
        const Rows lrow{lam, lam, B, B, s->N};
        if (diag_w) launch_diag_lambda(prow, lrow, s->n, diag_w, s->stream);
        else launch_apply_pauli_sum(prow, lrow, s->n, dterms, n_obs, dcoeff, s->stream, z_only_terms(obs, n_obs));
        launch_inner(prow, lrow, s->n, rscratch, d_loss, s->stream);

        const Rows both{s->psi, lam, B, 2 * B, s->N};
        uint64_t cur = 0;
        for (int i = n_ops - 1; i >= 0; --i) {
            const sv_op& op = ops[i];
            const OpInfo& oi = info[i];
            const int D = 1 << oi.k;
            if (oi.np == 0) {
                cd m[16], md[16];
                op_matrix(op, oi, params, m);
                dagger(oi.k, m, md);
                dispatch(both, oi.k, op.targets, op.n_controls, op.controls, md, s->stream);
                continue;
            }
            // rows whose parameters of this op are all equal share one launch
            const bool op_rows = per_row && !same_params_all_rows(op, oi, params, params_batch_stride, B);
            const int nrl = op_rows ? B : 1;
            for (int rl = 0; rl < nrl; ++rl) {
                const double* pr = params + (op_rows ? rl * params_batch_stride : 0);
                double prm[3];
                op_params(op, oi, pr, prm);
                cd m[16], md[16];
                kind_matrix(op.kind, prm, m);
                dagger(oi.k, m, md);
                AdjLaunch a{};
                if (op_rows) {
                    a.psi = one_row(s, s->psi, rl);
                    a.lam = one_row(s, lam, rl);
                } else {
                    a.psi = prow;
                    a.lam = lrow;
                }
                a.k = oi.k;
                for (int j = 0; j < oi.k; ++j) a.targets[j] = op.targets[j];
                a.nc = op.n_controls;
                for (int j = 0; j < op.n_controls; ++j) a.controls[j] = op.controls[j];
                for (int q = 0; q < D * D; ++q) a.uinv[q] = f2(md[q]);
                a.nd = oi.np;
                for (int d = 0; d < oi.np; ++d) {
                    cd dm[16];
                    kind_dmatrix(op.kind, prm, d, dm);
                    for (int r = 0; r < D; ++r)
                        for (int c = 0; c < D; ++c) {
                            cd acc = 0.0;
                            for (int j = 0; j < D; ++j) acc += dm[r * D + j] * md[j * D + c];
                            a.g[d][r * D + c] = make_double2(acc.real(), acc.imag());
                        }
                }
                a.grid = G;
                launch_adj_step(a, part + cur * G, s->stream);
                const int rows_here = op_rows ? 1 : B;
                for (int r = 0; r < rows_here; ++r)
                    for (int d = 0; d < oi.np; ++d) slots.push_back(Slot{op_rows ? rl : r, op.param[d]});
                cur += (uint64_t)rows_here * oi.np;
            }
        }
        if (cur > 0) launch_sum_slots(part, G, (int)cur, d_slots, s->stream);
        launch_drift(prow, s->n, rscratch, d_drift, s->stream);
        SV_HIP(hipMemcpyAsync(s->hout, s->dout, (std::max<uint64_t>(nslot_max, 1) + 3ull * B) * sizeof(double),
                              hipMemcpyDeviceToHost, s->stream));
        SV_HIP(hipStreamSynchronize(s->stream));
        const double* h_slots = s->hout;
        const double* h_loss = s->hout + std::max<uint64_t>(nslot_max, 1);
        const double* h_drift = h_loss + 2ull * B;
        if (n_params > 0) std::fill(grad_out, grad_out + (size_t)B * n_params, 0.0);
        // slots were pushed in reverse gate order; accumulate in that fixed order
        for (uint64_t q = 0; q < cur; ++q) grad_out[(size_t)slots[q].row * n_params + slots[q].param] += 2.0 * h_slots[q];
        for (int r = 0; r < B; ++r) {
            if (loss_out) loss_out[r] = h_loss[2 * r];
            if (drift_out) drift_out[r] = std::sqrt(std::max(0.0, h_drift[r]));
        }
    });
}


// The backward over blocks of gates on at most lb qubits (one sweep per
// block, k_adj_block). Same quantities as adjoint_impl, gate by gate.
sv_status adjoint_blocked_impl(sv_state s, const sv_op* ops, int n_ops, const double* params,
                               int64_t params_batch_stride, int n_params, const sv_pauli_term* obs, int n_obs,
                               const double* coeff_rows, int lb, void* lambda_buffer, double* grad_out,
                               double* loss_out, double* drift_out, const double* diag_w = nullptr)
{
    return guarded([&] {
        check_state(s);
        need(lb >= 3 && lb <= 5, SV_ERR_INVALID_ARGUMENT, "block width must be 3, 4 or 5");
        need(s->n >= lb, SV_ERR_INVALID_ARGUMENT, "the state has fewer qubits than the block width");
        need(n_ops >= 0 && (n_ops == 0 || ops != nullptr), SV_ERR_INVALID_ARGUMENT, "ops is NULL");
        need(n_params >= 0 && (n_params == 0 || params != nullptr), SV_ERR_INVALID_ARGUMENT, "params is NULL");
        need(n_params == 0 || grad_out != nullptr, SV_ERR_INVALID_ARGUMENT, "grad_out is NULL");
        need(params_batch_stride >= 0, SV_ERR_INVALID_ARGUMENT, "negative params stride");
        if (!diag_w) check_terms(s->n, obs, n_obs);
        std::vector<OpInfo> info(n_ops);
        std::vector<uint64_t> masks(n_ops);
        for (int i = 0; i < n_ops; ++i) {
            const sv_op& op = ops[i];
            info[i] = check_op(s->n, op, n_params);
            need(op.kind != SV_MATRIX || info[i].k <= 2, SV_ERR_UNSUPPORTED, "matrix ops of more than two targets");
            need(info[i].np <= (info[i].k == 1 ? 3 : 1), SV_ERR_UNSUPPORTED, "two-target kinds with several parameters");
            need(info[i].k == 1 || info[i].np == 0 || op.kind == SV_RXX || op.kind == SV_RYY || op.kind == SV_RZZ,
                 SV_ERR_UNSUPPORTED, "parameterised two-target ops other than RXX, RYY, RZZ");
            for (int j = 0; j < info[i].k; ++j) masks[i] |= 1ull << op.targets[j];
            for (int j = 0; j < op.n_controls; ++j) masks[i] |= 1ull << op.controls[j];
            need(__builtin_popcountll(masks[i]) <= lb, SV_ERR_UNSUPPORTED,
                 "op " + std::to_string(i) + " acts on more qubits than the block width");
        }
        check_not_capturing(s->stream);

        const int B = s->batch;
        const bool per_row = params_batch_stride != 0 && B > 1;
        float2* lam = nullptr;
        ensure_lambda(s, lambda_buffer, &lam);
        PauliTermDev* dterms = nullptr;
        const double* dcoeff = nullptr;
        if (!diag_w) upload_terms(s, obs, n_obs, coeff_rows, B, &dterms, &dcoeff);

        // ---- plan on the host: launches (block, row set, gate range) and their gate tables
        struct Launch {
            int row;                      // -1: all rows
            std::array<int, kAdjBlockMaxBits> q;
            size_t first;                 // first entry in the gate table
            int ngates;
            int nslots;
            std::vector<int> slot_param;  // parameter of each slot
        };
        std::vector<Launch> launches;
        std::vector<AdjBlockGate> table;
        const std::vector<GateBlock> blocks = plan_gate_blocks(masks, lb);
        for (int bi = (int)blocks.size() - 1; bi >= 0; --bi) {
            const GateBlock& gb = blocks[bi];
            // local qubits: the block's, padded with the lowest free qubits, ascending
            uint64_t used = 0;
            for (int q : gb.qs) used |= 1ull << q;
            for (int q = 0; q < s->n && __builtin_popcountll(used) < lb; ++q) used |= 1ull << q;
            std::array<int, kAdjBlockMaxBits> lq{};
            int nq = 0;
            for (int q = 0; q < s->n; ++q)
                if ((used >> q) & 1) lq[nq++] = q;
            auto local = [&](int q) {
                for (int i = 0; i < lb; ++i)
                    if (lq[i] == q) return i;
                return -1;
            };
            bool rows_differ = false;
            if (per_row)
                for (int gi : gb.gates)
                    if (info[gi].np > 0 && !same_params_all_rows(ops[gi], info[gi], params, params_batch_stride, B))
                        rows_differ = true;
            const int nrl = rows_differ ? B : 1;
            for (int rl = 0; rl < nrl; ++rl) {
                const double* prow = params + (rows_differ ? rl * params_batch_stride : 0);
                Launch L{};
                L.row = rows_differ ? rl : -1;
                L.q = lq;
                L.first = table.size();
                auto close = [&] {
                    if (L.ngates > 0) launches.push_back(L);
                    L.first = table.size();
                    L.ngates = 0;
                    L.nslots = 0;
                    L.slot_param.clear();
                };
                for (int t = (int)gb.gates.size() - 1; t >= 0; --t) {
                    const int gi = gb.gates[t];
                    const sv_op& op = ops[gi];
                    const OpInfo& oi = info[gi];
                    if (L.nslots + oi.np > kAdjBlockMaxSlots) close();
                    const int D = 1 << oi.k;
                    double prm[3];
                    op_params(op, oi, prow, prm);
                    cd m[16], md[16];
                    op_matrix(op, oi, prow, m);
                    dagger(oi.k, m, md);
                    AdjBlockGate g{};
                    g.nt = oi.k;
                    g.t0 = local(op.targets[0]);
                    g.t1 = oi.k == 2 ? local(op.targets[1]) : 0;
                    for (int j = 0; j < op.n_controls; ++j) g.cmask |= 1 << local(op.controls[j]);
                    for (int q = 0; q < D * D; ++q) g.u[q] = f2(md[q]);
                    bool diag = true;
                    for (int r = 0; r < D; ++r)
                        for (int c = 0; c < D; ++c)
                            if (r != c && md[r * D + c] != cd(0.0)) diag = false;
                    const bool exch = oi.k == 1 && md[0] == cd(0.0) && md[3] == cd(0.0) && md[1] == cd(1.0) &&
                                      md[2] == cd(1.0);
                    g.form = exch ? 2 : (diag ? 1 : 0);
                    g.nd = oi.np;
                    switch (op.kind) {
                    case SV_RX: g.pauli = 1; break;
                    case SV_RY: g.pauli = 2; break;
                    case SV_RZ: g.pauli = 3; break;
                    case SV_RXX: g.pauli = 4; break;
                    case SV_RYY: g.pauli = 5; break;
                    case SV_RZZ: g.pauli = 6; break;
                    default: g.pauli = 0; break;
                    }
                    for (int d = 0; d < oi.np; ++d) {
                        g.slot[d] = L.nslots++;
                        L.slot_param.push_back(op.param[d]);
                        if (g.pauli) continue;
                        cd dm[16];
                        kind_dmatrix(op.kind, prm, d, dm);
                        for (int r = 0; r < D; ++r)
                            for (int c = 0; c < D; ++c) {
                                cd acc = 0.0;
                                for (int j = 0; j < D; ++j) acc += dm[r * D + j] * md[j * D + c];
                                g.g[d][r * D + c] = make_double2(acc.real(), acc.imag());
                            }
                    }
                    table.push_back(g);
                    ++L.ngates;
                }
                close();
            }
        }

        // ---- device buffers: gate table, partials, slot sums
        const int G = adj_block_grid(s->n, lb);
        uint64_t nslot_total = 0, part_max = 1;
        for (const Launch& L : launches) {
            const int rows_here = L.row < 0 ? B : 1;
            nslot_total += (uint64_t)rows_here * L.nslots;
            part_max = std::max<uint64_t>(part_max, (uint64_t)rows_here * L.nslots * 4 * G);
        }
        const uint64_t red = std::max<uint64_t>(inner_parts(s->n, B), drift_parts(s->n, B));
        const uint64_t table_doubles = (table.size() * sizeof(AdjBlockGate) + 7) / 8 + 2;
        const uint64_t table_at = (part_max + red + 1) & ~1ull;       // 16-byte aligned
        ensure_scratch(s, table_at + table_doubles);
        double* part = s->scratch;
        double* rscratch = s->scratch + part_max;
        AdjBlockGate* dtable = reinterpret_cast<AdjBlockGate*>(s->scratch + table_at);
        if (!table.empty())
            SV_HIP(hipMemcpyAsync(dtable, table.data(), table.size() * sizeof(AdjBlockGate), hipMemcpyHostToDevice,
                                  s->stream));
        const uint64_t nout = std::max<uint64_t>(nslot_total, 1) + 3ull * B;
        ensure_dout(s, nout + 2ull * B);
        double* d_slots = s->dout;
        double* d_loss = s->dout + std::max<uint64_t>(nslot_total, 1);
        double* d_drift = d_loss + 2ull * B;

        const Rows prow{s->psi, s->psi, B, B, s->N};
        const Rows lrow{lam, lam, B, B, s->N};
        if (diag_w) launch_diag_lambda(prow, lrow, s->n, diag_w, s->stream);
        else launch_apply_pauli_sum(prow, lrow, s->n, dterms, n_obs, dcoeff, s->stream, z_only_terms(obs, n_obs));
        launch_inner(prow, lrow, s->n, rscratch, d_loss, s->stream);

        struct Slot { int row; int param; };
        std::vector<Slot> slots;
        slots.reserve(nslot_total);
        uint64_t cur = 0;
        for (const Launch& L : launches) {
            AdjBlockLaunch a{};
            if (L.row >= 0) {
                a.psi = one_row(s, s->psi, L.row);
                a.lam = one_row(s, lam, L.row);
            } else {
                a.psi = prow;
                a.lam = lrow;
            }
            for (int i = 0; i < lb; ++i) {
                a.q[i] = L.q[i];
                a.qbit[i] = 1ull << L.q[i];
            }
            a.lb = lb;
            a.ngates = L.ngates;
            a.gates = dtable + L.first;
            a.nslots = L.nslots;
            a.grid = G;
            launch_adj_block(a, part, s->stream);
            const int rows_here = L.row < 0 ? B : 1;
            if (L.nslots > 0) {
                launch_sum_slots(part, 4 * G, rows_here * L.nslots, d_slots + cur, s->stream);
                for (int r = 0; r < rows_here; ++r)
                    for (int q = 0; q < L.nslots; ++q) slots.push_back(Slot{L.row >= 0 ? L.row : r, L.slot_param[q]});
                cur += (uint64_t)rows_here * L.nslots;
            }
        }
        launch_drift(prow, s->n, rscratch, d_drift, s->stream);
        SV_HIP(hipMemcpyAsync(s->hout, s->dout, nout * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        SV_HIP(hipStreamSynchronize(s->stream));
        const double* h_slots = s->hout;
        const double* h_loss = s->hout + std::max<uint64_t>(nslot_total, 1);
        const double* h_drift = h_loss + 2ull * B;
        if (n_params > 0) std::fill(grad_out, grad_out + (size_t)B * n_params, 0.0);
        for (uint64_t q = 0; q < cur; ++q) grad_out[(size_t)slots[q].row * n_params + slots[q].param] += 2.0 * h_slots[q];
        for (int r = 0; r < B; ++r) {
            if (loss_out) loss_out[r] = h_loss[2 * r];
            if (drift_out) drift_out[r] = std::sqrt(std::max(0.0, h_drift[r]));
        }
    });
}

}  // namespace

namespace {

// 16 x 16 embedding of a gate on a block's local bits: targets tl[0..k-1]
// (tl[0] the most significant bit of m's index), controls cm; columns whose
// control bits are not all 1 get the identity (id) or zero.
void embed16(const cd* m, int k, const int* tl, int cm, bool id, cd* E)
{
    std::fill(E, E + 256, cd(0.0));
    const int D = 1 << k;
    for (int c = 0; c < 16; ++c) {
        if ((c & cm) != cm) {
            if (id) E[c * 16 + c] = 1.0;
            continue;
        }
        int sin = 0, clr = c;
        for (int t = 0; t < k; ++t) {
            sin |= ((c >> tl[t]) & 1) << (k - 1 - t);
            clr &= ~(1 << tl[t]);
        }
        for (int so = 0; so < D; ++so) {
            int r = clr;
            for (int t = 0; t < k; ++t)
                if ((so >> (k - 1 - t)) & 1) r |= 1 << tl[t];
            E[r * 16 + c] += m[so * D + sin];
        }
    }
}

// A block's embedded gate as its nonzero entries: at most four per column
// for a gate on at most two targets. Products with it cost 16 complex
// multiply-adds per entry instead of 256 per column. Complex products are
// written out in real arithmetic (the library's complex operator* keeps the
// C99 special-value rules and is many times slower).
struct Sp16 {
    int n = 0;
    uint8_t r[64], c[64];
    cd v[64];
};

void sparse16(const cd* E, Sp16& S)
{
    S.n = 0;
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c)
            if (E[r * 16 + c] != cd(0.0)) {
                need(S.n < 64, SV_ERR_UNSUPPORTED, "embedded gate has more than 64 entries");
                S.r[S.n] = (uint8_t)r;
                S.c[S.n] = (uint8_t)c;
                S.v[S.n++] = E[r * 16 + c];
            }
}

// C += v a, over a row of 16
inline void axpy16(cd v, const cd* a, cd* o)
{
    const double vr = v.real(), vi = v.imag();
    for (int c = 0; c < 16; ++c) {
        const double ar = a[c].real(), ai = a[c].imag();
        o[c] = cd(o[c].real() + vr * ar - vi * ai, o[c].imag() + vr * ai + vi * ar);
    }
}

// C = E A
void sp_left(const Sp16& E, const cd* A, cd* C)
{
    std::fill(C, C + 256, cd(0.0));
    for (int k = 0; k < E.n; ++k) axpy16(E.v[k], A + E.c[k] * 16, C + E.r[k] * 16);
}

// C = E^* A
void sp_adj_left(const Sp16& E, const cd* A, cd* C)
{
    std::fill(C, C + 256, cd(0.0));
    for (int k = 0; k < E.n; ++k) axpy16(std::conj(E.v[k]), A + E.r[k] * 16, C + E.c[k] * 16);
}

// C = A E
void sp_right(const cd* A, const Sp16& E, cd* C)
{
    std::fill(C, C + 256, cd(0.0));
    for (int k = 0; k < E.n; ++k) {
        const int j = E.r[k], c = E.c[k];
        const double vr = E.v[k].real(), vi = E.v[k].imag();
        for (int r = 0; r < 16; ++r) {
            const double ar = A[r * 16 + j].real(), ai = A[r * 16 + j].imag();
            C[r * 16 + c] = cd(C[r * 16 + c].real() + ar * vr - ai * vi, C[r * 16 + c].imag() + ar * vi + ai * vr);
        }
    }
}

// C = A B^*
void mm16_adj(const cd* A, const cd* B, cd* C)
{
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c) {
            double re = 0.0, im = 0.0;
            for (int j = 0; j < 16; ++j) {
                const double ar = A[r * 16 + j].real(), ai = A[r * 16 + j].imag();
                const double br = B[c * 16 + j].real(), bi = -B[c * 16 + j].imag();
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            C[r * 16 + c] = cd(re, im);
        }
}

// Operand fragments of the real form [[Re M, -Im M], [Im M, Re M]] for the
// FP32 product of k_adj_mfma: lane i + 32 (c >> 3), entry 2 (c & 7) + ci
// holds row i (output component i & 1 of amplitude 8 ((i >> 2) & 1) +
// 2 (i >> 3) + ((i >> 1) & 1)) against input column (amplitude c,
// component ci).
void mfma_fragments(const cd* M, float* frag)
{
    for (int c = 0; c < 16; ++c)
        for (int i = 0; i < 32; ++i) {
            const int jo = 8 * ((i >> 2) & 1) + 2 * (i >> 3) + ((i >> 1) & 1);
            const cd e = M[jo * 16 + c];
            for (int ci = 0; ci < 2; ++ci) {
                const double v = (i & 1) == 0 ? (ci == 0 ? e.real() : -e.imag()) : (ci == 0 ? e.imag() : e.real());
                frag[(i + 32 * (c >> 3)) * 16 + 2 * (c & 7) + ci] = (float)v;
            }
        }
}

// The blocked backward on the matrix cores (k_adj_mfma): blocks of gates on
// at most four qubits; per block one sweep for the correlation S and the
// un-apply, then each derivative as 2 Re Tr(X_k S) on the host.
sv_status adjoint_mfma_impl(sv_state s, const sv_op* ops, int n_ops, const double* params,
                            int64_t params_batch_stride, int n_params, const sv_pauli_term* obs, int n_obs,
                            const double* coeff_rows, void* lambda_buffer, double* grad_out, double* loss_out,
                            double* drift_out, const double* diag_w)
{
    return guarded([&] {
        constexpr int lb = 4;
        constexpr int kRecurRows = 4;
        check_state(s);
        need(s->n >= 9, SV_ERR_UNSUPPORTED, "the matrix-core adjoint needs at least 9 qubits");
        need(n_ops >= 0 && (n_ops == 0 || ops != nullptr), SV_ERR_INVALID_ARGUMENT, "ops is NULL");
        need(n_params >= 0 && (n_params == 0 || params != nullptr), SV_ERR_INVALID_ARGUMENT, "params is NULL");
        need(n_params == 0 || grad_out != nullptr, SV_ERR_INVALID_ARGUMENT, "grad_out is NULL");
        need(params_batch_stride >= 0, SV_ERR_INVALID_ARGUMENT, "negative params stride");
        if (!diag_w) check_terms(s->n, obs, n_obs);
        std::vector<OpInfo> info(n_ops);
        std::vector<uint64_t> masks(n_ops);
        for (int i = 0; i < n_ops; ++i) {
            const sv_op& op = ops[i];
            info[i] = check_op(s->n, op, n_params);
            for (int j = 0; j < info[i].k; ++j) masks[i] |= 1ull << op.targets[j];
            for (int j = 0; j < op.n_controls; ++j) masks[i] |= 1ull << op.controls[j];
            need(__builtin_popcountll(masks[i]) <= lb, SV_ERR_UNSUPPORTED,
                 "op " + std::to_string(i) + " acts on more than four qubits");
        }
        check_not_capturing(s->stream);

        const int B = s->batch;
        const bool per_row = params_batch_stride != 0 && B > 1;
        float2* lam = nullptr;
        ensure_lambda(s, lambda_buffer, &lam);
        PauliTermDev* dterms = nullptr;
        const double* dcoeff = nullptr;
        if (!diag_w) upload_terms(s, obs, n_obs, coeff_rows, B, &dterms, &dcoeff);

        // ---- plan on the host: one launch per block over every row; a block
        // holding gates whose parameters differ between rows gets its product
        // (fragments) per row. The derivatives come either from X_k formed
        // on the host while the GPU sweeps (a block shared by more than
        // kRecurRows rows: one X_k serves every row), or from S itself once
        // its copy is back, S_t = W_t^* S W_t stepped down the gates
        // (Tr(X_k S) = Tr(G_k S_t)): a few times cheaper per row, but only
        // after that block's sweep.
        struct Deriv { int param; size_t x; };      // X_k at xs[x * 256]
        struct Launch {
            int q[4];
            const GateBlock* gb;
            std::vector<int> tl, cm;                 // local targets (2 per gate), control masks
            int nfr;                                 // 1: one product for all rows; B: one per row
            bool recur;                              // derivatives by the S_t recursion
            size_t frag_at;                          // first fragment block (1024 floats each)
            std::vector<size_t> e_at;                // per product: E of its gates at es[e_at + t]
            std::vector<Deriv> d;                    // shared product: its X_k
        };
        std::vector<Launch> launches;
        std::vector<Sp16> es;
        std::vector<cd> xs;
        const std::vector<GateBlock> blocks = plan_gate_blocks(masks, lb);
        std::vector<cd> U(256), T1(256), T2(256), W(256), Ed(256);
        Sp16 Gs;
        // G = dG_k G_k^* of parameter d of gate t, embedded in the block
        auto gate_derivative = [&](const Launch& L, int t, const double* prow, int d, Sp16& out) {
            const sv_op& op = ops[L.gb->gates[t]];
            const OpInfo& oi = info[L.gb->gates[t]];
            const int D = 1 << oi.k;
            double prm[3];
            op_params(op, oi, prow, prm);
            cd m[16], md[16], dm[16], g[16];
            op_matrix(op, oi, prow, m);
            dagger(oi.k, m, md);
            kind_dmatrix(op.kind, prm, d, dm);
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) {
                    double re = 0.0, im = 0.0;
                    for (int j = 0; j < D; ++j) {
                        const cd x = dm[r * D + j], y = md[j * D + c];
                        re += x.real() * y.real() - x.imag() * y.imag();
                        im += x.real() * y.imag() + x.imag() * y.real();
                    }
                    g[r * D + c] = cd(re, im);
                }
            embed16(g, oi.k, &L.tl[2 * t], L.cm[t], false, Ed.data());
            sparse16(Ed.data(), out);
        };
        // structure of every launch (its matrices come later, chunk by chunk)
        size_t n_frag = 0, n_es = 0;
        for (int bi = (int)blocks.size() - 1; bi >= 0; --bi) {
            const GateBlock& gb = blocks[bi];
            uint64_t used = 0;
            for (int q : gb.qs) used |= 1ull << q;
            for (int q = 0; q < s->n && __builtin_popcountll(used) < lb; ++q) used |= 1ull << q;
            int lq[4], nq = 0;
            for (int q = 0; q < s->n; ++q)
                if ((used >> q) & 1) lq[nq++] = q;
            auto local = [&](int q) {
                for (int i = 0; i < lb; ++i)
                    if (lq[i] == q) return i;
                return -1;
            };
            bool rows_differ = false;
            if (per_row)
                for (int gi : gb.gates)
                    if (info[gi].np > 0 && !same_params_all_rows(ops[gi], info[gi], params, params_batch_stride, B))
                        rows_differ = true;
            const int ng = (int)gb.gates.size();
            Launch L{};
            for (int i = 0; i < 4; ++i) L.q[i] = lq[i];
            L.gb = &gb;
            L.tl.assign(ng * 2, 0);
            L.cm.assign(ng, 0);
            for (int t = 0; t < ng; ++t) {
                const sv_op& op = ops[gb.gates[t]];
                L.tl[2 * t] = local(op.targets[0]);
                L.tl[2 * t + 1] = info[gb.gates[t]].k == 2 ? local(op.targets[1]) : 0;
                for (int j = 0; j < op.n_controls; ++j) L.cm[t] |= 1 << local(op.controls[j]);
            }
            L.nfr = rows_differ ? B : 1;
            L.recur = rows_differ || B <= kRecurRows;
            L.frag_at = n_frag;
            n_frag += L.nfr;
            for (int rl = 0; rl < L.nfr; ++rl) {
                L.e_at.push_back(n_es);
                n_es += ng;
            }
            launches.push_back(std::move(L));
        }
        es.resize(n_es);
        // the embedded gates E of launch L and its products' fragments
        auto form_products = [&](const Launch& L, float* frag) {
            const int ng = (int)L.gb->gates.size();
            for (int rl = 0; rl < L.nfr; ++rl) {
                const double* prow = params + (L.nfr > 1 ? rl * params_batch_stride : 0);
                const size_t ea = L.e_at[rl];
                // U_B = E_last ... E_first; the kernel applies M = U_B^*
                for (int q = 0; q < 256; ++q) U[q] = (q % 17 == 0) ? 1.0 : 0.0;
                for (int t = 0; t < ng; ++t) {
                    const sv_op& op = ops[L.gb->gates[t]];
                    const OpInfo& oi = info[L.gb->gates[t]];
                    cd m[16];
                    op_matrix(op, oi, prow, m);
                    embed16(m, oi.k, &L.tl[2 * t], L.cm[t], true, Ed.data());
                    sparse16(Ed.data(), es[ea + t]);
                    sp_left(es[ea + t], U.data(), T1.data());
                    U.swap(T1);
                }
                for (int r = 0; r < 16; ++r)
                    for (int c = 0; c < 16; ++c) T1[r * 16 + c] = std::conj(U[c * 16 + r]);
                mfma_fragments(T1.data(), frag + (size_t)rl * 1024);
            }
        };
        // X_k = W_k (dG_k G_k^*) W_k^*, W_k the gates after k (host, FP64)
        auto form_derivatives = [&] {
            for (Launch& L : launches) {
                if (L.recur) continue;
                const int ng = (int)L.gb->gates.size();
                const size_t ea = L.e_at[0];
                for (int q = 0; q < 256; ++q) W[q] = (q % 17 == 0) ? 1.0 : 0.0;
                for (int t = ng - 1; t >= 0; --t) {
                    const int gi = L.gb->gates[t];
                    for (int d = 0; d < info[gi].np; ++d) {
                        gate_derivative(L, t, params, d, Gs);
                        sp_right(W.data(), Gs, T1.data());
                        mm16_adj(T1.data(), W.data(), T2.data());
                        L.d.push_back(Deriv{ops[gi].param[d], xs.size() / 256});
                        xs.insert(xs.end(), T2.begin(), T2.end());
                    }
                    sp_right(W.data(), es[ea + t], T1.data());
                    W.swap(T1);
                }
            }
        };

        // ---- device buffers: fragments, the waves' S parts, S per launch and row
        const AdjMfmaShape shape = adj_mfma_shape(s->n, B);
        const int grid = shape.grid;
        const uint64_t spart_max = std::max<uint64_t>(1, adj_mfma_part_doubles(grid, B));
        const uint64_t s_total = (uint64_t)launches.size() * B * 1024;
        const uint64_t red = std::max<uint64_t>(inner_parts(s->n, B), drift_parts(s->n, B));
        const uint64_t frag_doubles = n_frag * 512 + 2;
        const uint64_t frag_at = (spart_max + red + 1) & ~1ull;
        ensure_scratch(s, frag_at + frag_doubles);
        ensure_hstage(s, n_frag * 1024);
        double* spart = s->scratch;
        double* rscratch = s->scratch + spart_max;
        float* dfrag = reinterpret_cast<float*>(s->scratch + frag_at);
        float* hfrag = s->hstage;
        const uint64_t s_room = std::max<uint64_t>(s_total, 1);
        const uint64_t nout = s_room + 3ull * B;
        ensure_dout(s, nout + 2ull * B);
        double* d_s = s->dout;
        double* d_loss = s->dout + s_room;
        double* d_drift = d_loss + 2ull * B;
        const double* h_s = s->hout;
        const double* h_loss = s->hout + s_room;
        const double* h_drift = h_loss + 2ull * B;

        const Rows prow{s->psi, s->psi, B, B, s->N};
        const Rows lrow{lam, lam, B, B, s->N};
        if (diag_w) launch_diag_lambda(prow, lrow, s->n, diag_w, s->stream);
        else launch_apply_pauli_sum(prow, lrow, s->n, dterms, n_obs, dcoeff, s->stream, z_only_terms(obs, n_obs));
        launch_inner(prow, lrow, s->n, rscratch, d_loss, s->stream);

        // chunks of launches: the host forms a chunk's products while the
        // GPU runs the one before, and traces a chunk's S as soon as its copy
        // is back
        const int nl = (int)launches.size();
        const int n_chunks = std::max(1, std::min(kAmEvents, (nl + 3) / 4));
        ensure_events(s);
        auto chunk_begin = [&](int c) { return (int)((int64_t)nl * c / n_chunks); };
        for (int c = 0; c < n_chunks; ++c) {
            const int l0 = chunk_begin(c), l1 = chunk_begin(c + 1);
            if (l0 == l1) continue;
            for (int li = l0; li < l1; ++li) form_products(launches[li], hfrag + launches[li].frag_at * 1024);
            const size_t f0 = launches[l0].frag_at, f1 = launches[l1 - 1].frag_at + launches[l1 - 1].nfr;
            SV_HIP(hipMemcpyAsync(dfrag + f0 * 1024, hfrag + f0 * 1024, (f1 - f0) * 1024 * sizeof(float),
                                  hipMemcpyHostToDevice, s->stream));
            for (int li = l0; li < l1; ++li) {
                const Launch& L = launches[li];
                AdjMfmaLaunch a{};
                a.psi = prow;
                a.lam = lrow;
                a.N = s->N;
                for (int i = 0; i < 4; ++i) a.q[i] = L.q[i];
                a.frag = dfrag + L.frag_at * 1024;
                a.frag_stride = L.nfr > 1 ? 1024 : 0;
                a.spart = spart;
                a.grid = grid;
                a.gpw = shape.gpw;
                launch_adj_mfma(a, B, d_s + (size_t)li * B * 1024, s->stream);
            }
            SV_HIP(hipMemcpyAsync(s->hout + (size_t)l0 * B * 1024, d_s + (size_t)l0 * B * 1024,
                                  (size_t)(l1 - l0) * B * 1024 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
            SV_HIP(hipEventRecord(s->events[c], s->stream));
        }
        launch_drift(prow, s->n, rscratch, d_drift, s->stream);
        SV_HIP(hipMemcpyAsync(s->hout + s_room, d_loss, 3ull * B * sizeof(double), hipMemcpyDeviceToHost,
                              s->stream));
        form_derivatives();        // while the sweeps run
        if (n_params > 0) std::fill(grad_out, grad_out + (size_t)B * n_params, 0.0);
        // derivatives in launch (reverse block) order, then gate order
        std::vector<cd> S(256);
        for (int c = 0; c < n_chunks; ++c) {
            const int l0 = chunk_begin(c), l1 = chunk_begin(c + 1);
            if (l0 == l1) continue;
            SV_HIP(hipEventSynchronize(s->events[c]));
            for (int li = l0; li < l1; ++li) {
                const Launch& L = launches[li];
                const int ng = (int)L.gb->gates.size();
                for (int r = 0; r < B; ++r) {
                    const double* sr = h_s + ((size_t)li * B + r) * 1024;     // S_real[32][32]
                    for (int b = 0; b < 16; ++b)
                        for (int a2 = 0; a2 < 16; ++a2)
                            S[b * 16 + a2] = cd(sr[b * 32 + a2] + sr[(16 + b) * 32 + 16 + a2],
                                                sr[(16 + b) * 32 + a2] - sr[b * 32 + 16 + a2]);
                    double* g = grad_out + (size_t)r * n_params;
                    if (!L.recur) {
                        for (const Deriv& dv : L.d) {
                            const cd* X = &xs[dv.x * 256];
                            double tr = 0.0;       // Re Tr(X S)
                            for (int a2 = 0; a2 < 16; ++a2)
                                for (int b = 0; b < 16; ++b) {
                                    const cd x = X[a2 * 16 + b], y = S[b * 16 + a2];
                                    tr += x.real() * y.real() - x.imag() * y.imag();
                                }
                            g[dv.param] += 2.0 * tr;
                        }
                        continue;
                    }
                    const double* prow_r = params + (L.nfr > 1 ? r * params_batch_stride : 0);
                    const size_t ea = L.e_at[L.nfr > 1 ? r : 0];
                    for (int t = ng - 1; t >= 0; --t) {       // S holds S_t = W_t^* S W_t
                        const int gi = L.gb->gates[t];
                        for (int d = 0; d < info[gi].np; ++d) {
                            gate_derivative(L, t, prow_r, d, Gs);
                            double tr = 0.0;       // Re Tr(G S_t)
                            for (int k = 0; k < Gs.n; ++k) {
                                const cd x = Gs.v[k], y = S[Gs.c[k] * 16 + Gs.r[k]];
                                tr += x.real() * y.real() - x.imag() * y.imag();
                            }
                            g[ops[gi].param[d]] += 2.0 * tr;
                        }
                        if (t > 0) {
                            sp_right(S.data(), es[ea + t], T1.data());
                            sp_adj_left(es[ea + t], T1.data(), S.data());
                        }
                    }
                }
            }
        }
        SV_HIP(hipStreamSynchronize(s->stream));
        for (int r = 0; r < B; ++r) {
            if (loss_out) loss_out[r] = h_loss[2 * r];
            if (drift_out) drift_out[r] = std::sqrt(std::max(0.0, h_drift[r]));
        }
    });
}

}  // namespace

extern "C" {

sv_status sv_adjoint_grad(sv_state s, const sv_op* ops, int n_ops, const double* params,
                          int64_t params_batch_stride, int n_params, const sv_pauli_term* obs, int n_obs,
                          void* lambda_buffer, double* grad_out, double* loss_out, double* drift_out)
{
    return adjoint_impl(s, ops, n_ops, params, params_batch_stride, n_params, obs, n_obs, nullptr, lambda_buffer,
                        grad_out, loss_out, drift_out);
}

sv_status sv_adjoint_grad_weighted(sv_state s, const sv_op* ops, int n_ops, const double* params,
                                   int64_t params_batch_stride, int n_params, const sv_pauli_term* obs, int n_obs,
                                   const double* coeff_rows, void* lambda_buffer, double* grad_out,
                                   double* loss_out, double* drift_out)
{
    if (coeff_rows == nullptr) {
        g_last_error = "coeff_rows is NULL";
        return SV_ERR_INVALID_ARGUMENT;
    }
    return adjoint_impl(s, ops, n_ops, params, params_batch_stride, n_params, obs, n_obs, coeff_rows, lambda_buffer,
                        grad_out, loss_out, drift_out);
}

sv_status sv_adjoint_grad_mfma(sv_state s, const sv_op* ops, int n_ops, const double* params,
                               int64_t params_batch_stride, int n_params, const sv_pauli_term* obs, int n_obs,
                               const double* coeff_rows, void* lambda_buffer, double* grad_out, double* loss_out,
                               double* drift_out)
{
    return adjoint_mfma_impl(s, ops, n_ops, params, params_batch_stride, n_params, obs, n_obs, coeff_rows,
                             lambda_buffer, grad_out, loss_out, drift_out, nullptr);
}

sv_status sv_adjoint_grad_diag(sv_state s, const sv_op* ops, int n_ops, const double* params,
                               int64_t params_batch_stride, int n_params, const double* dev_weights,
                               int block_qubits, void* lambda_buffer, double* grad_out, double* loss_out,
                               double* drift_out)
{
    if (dev_weights == nullptr) {
        set_last_error("dev_weights is NULL");
        return SV_ERR_INVALID_ARGUMENT;
    }
    if (block_qubits == SV_ADJOINT_MFMA)
        return adjoint_mfma_impl(s, ops, n_ops, params, params_batch_stride, n_params, nullptr, 0, nullptr,
                                 lambda_buffer, grad_out, loss_out, drift_out, dev_weights);
    if (block_qubits == 0)
        return adjoint_impl(s, ops, n_ops, params, params_batch_stride, n_params, nullptr, 0, nullptr, lambda_buffer,
                            grad_out, loss_out, drift_out, dev_weights);
    return adjoint_blocked_impl(s, ops, n_ops, params, params_batch_stride, n_params, nullptr, 0, nullptr,
                                block_qubits, lambda_buffer, grad_out, loss_out, drift_out, dev_weights);
}

sv_status sv_adjoint_grad_blocked(sv_state s, const sv_op* ops, int n_ops, const double* params,
                                  int64_t params_batch_stride, int n_params, const sv_pauli_term* obs, int n_obs,
                                  const double* coeff_rows, int block_qubits, void* lambda_buffer, double* grad_out,
                                  double* loss_out, double* drift_out)
{
    return adjoint_blocked_impl(s, ops, n_ops, params, params_batch_stride, n_params, obs, n_obs, coeff_rows,
                                block_qubits, lambda_buffer, grad_out, loss_out, drift_out);
}

sv_status sv_sample_exact(sv_state s, int row, const double* dev_uniforms, int64_t n_shots, int64_t* dev_out)
{
    return guarded([&] {
        check_state(s);
        need(row >= 0 && row < s->batch, SV_ERR_INVALID_ARGUMENT, "row out of range");
        need(n_shots >= 0 && n_shots <= 2147483647ll, SV_ERR_INVALID_ARGUMENT, "n_shots must be 0..2^31-1");
        need(n_shots == 0 || (dev_uniforms != nullptr && dev_out != nullptr), SV_ERR_INVALID_ARGUMENT,
             "NULL device pointer");
        const size_t bytes = shot_scratch_bytes(s->n, n_shots);
        ensure_scratch(s, (bytes + sizeof(double) - 1) / sizeof(double));
        ShotLaunch a{};
        a.psi = s->psi + (uint64_t)row * s->N;
        a.n = s->n;
        a.u = dev_uniforms;
        a.shots = n_shots;
        a.out = dev_out;
        a.scratch = s->scratch;
        launch_sample_exact(a, s->stream);
    });
}

sv_status sv_sample_z_estimate(sv_state s, const int64_t* dev_indices, int64_t n_shots, double* dev_est)
{
    return guarded([&] {
        check_state(s);
        need(n_shots >= 0 && n_shots <= 2147483647ll, SV_ERR_INVALID_ARGUMENT, "n_shots must be 0..2^31-1");
        need(dev_est != nullptr && (n_shots == 0 || dev_indices != nullptr), SV_ERR_INVALID_ARGUMENT,
             "NULL device pointer");
        need(((uintptr_t)dev_indices & 7) == 0 && ((uintptr_t)dev_est & 7) == 0, SV_ERR_INVALID_ARGUMENT,
             "device arrays must be 8-byte aligned");
        ensure_scratch(s, (uint64_t)s->n + 1);
        launch_shot_zest(dev_indices, n_shots, s->n, s->scratch, dev_est, s->stream);
    });
}

sv_status sv_sample_gaussian(sv_state s, int row, const double* dev_normals, double shots, double* dev_y)
{
    return guarded([&] {
        check_state(s);
        need(row >= 0 && row < s->batch, SV_ERR_INVALID_ARGUMENT, "row out of range");
        need(shots > 0 && std::isfinite(shots), SV_ERR_INVALID_ARGUMENT, "shots must be positive");
        need(dev_normals != nullptr && dev_y != nullptr, SV_ERR_INVALID_ARGUMENT, "NULL device pointer");
        need(((uintptr_t)dev_normals & 15) == 0 && ((uintptr_t)dev_y & 15) == 0, SV_ERR_INVALID_ARGUMENT,
             "device arrays must be 16-byte aligned");
        ensure_scratch(s, gauss_scratch_doubles(s->n));
        GaussLaunch a{};
        a.psi = s->psi + (uint64_t)row * s->N;
        a.n = s->n;
        a.z = dev_normals;
        a.shots = shots;
        a.y = dev_y;
        a.scratch = s->scratch;
        launch_sample_gaussian(a, s->stream);
    });
}

namespace {

GaussZLaunch gauss_z_launch(sv_state s, int row, const double* dev_normals, double shots)
{
    check_state(s);
    need(row >= 0 && row < s->batch, SV_ERR_INVALID_ARGUMENT, "row out of range");
    need(shots > 0 && std::isfinite(shots), SV_ERR_INVALID_ARGUMENT, "shots must be positive");
    need(dev_normals != nullptr, SV_ERR_INVALID_ARGUMENT, "NULL device pointer");
    need(((uintptr_t)dev_normals & 15) == 0, SV_ERR_INVALID_ARGUMENT, "device arrays must be 16-byte aligned");
    ensure_scratch(s, gauss_z_scratch_doubles(s->n));
    GaussZLaunch a{};
    a.psi = s->psi + (uint64_t)row * s->N;
    a.n = s->n;
    a.z = dev_normals;
    a.shots = shots;
    a.scratch = s->scratch;
    return a;
}

}  // namespace

sv_status sv_gaussian_expval_z(sv_state s, int row, const double* dev_normals, double shots, double* est_out)
{
    return guarded([&] {
        need(est_out != nullptr, SV_ERR_INVALID_ARGUMENT, "est_out is NULL");
        GaussZLaunch a = gauss_z_launch(s, row, dev_normals, shots);
        check_not_capturing(s->stream);
        ensure_dout(s, (uint64_t)s->n);
        a.est = s->dout;
        launch_gauss_z(a, s->stream);
        SV_HIP(hipMemcpyAsync(s->hout, s->dout, (size_t)s->n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        SV_HIP(hipStreamSynchronize(s->stream));
        for (int i = 0; i < s->n; ++i) est_out[i] = s->hout[i];
    });
}

sv_status sv_gaussian_expval_z_backward(sv_state s, int row, const double* dev_normals, double shots,
                                        const double* upstream, double* dev_weights)
{
    return guarded([&] {
        need(upstream != nullptr, SV_ERR_INVALID_ARGUMENT, "upstream is NULL");
        need(dev_weights != nullptr, SV_ERR_INVALID_ARGUMENT, "dev_weights is NULL");
        GaussZLaunch a = gauss_z_launch(s, row, dev_normals, shots);
        for (int i = 0; i < s->n; ++i) {
            need(std::isfinite(upstream[i]), SV_ERR_INVALID_ARGUMENT, "upstream values must be finite");
            a.g[i] = upstream[i];
        }
        a.w = dev_weights;
        launch_gauss_z_backward(a, s->stream);
    });
}

sv_status sv_stream_copy(void* dst, const void* src, uint64_t bytes, void* stream)
{
    return guarded([&] {
        need(dst && src, SV_ERR_INVALID_ARGUMENT, "null pointer");
        need(bytes % 16 == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0 &&
                 (reinterpret_cast<uintptr_t>(src) & 15) == 0,
             SV_ERR_INVALID_ARGUMENT, "copy needs 16-byte aligned pointers and size");
        if (bytes) launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream));
    });
}

sv_status sv_sweep_order_tune(sv_state s, float* ms_out)
{
    return guarded([&] {
        check_state(s);
        check_not_capturing(s->stream);
        const int n = s->n;
        uint64_t mask = half_order_mask(n);
        if (ms_out)
            for (int i = 0; i < 2 * n; ++i) ms_out[i] = 0.0f;
        bool any = false;
        for (int t = 0; t < n; ++t) any = any || half_sweep_applies(n, t);
        if (!any) return;
        hipEvent_t ev[2];
        SV_HIP(hipEventCreate(&ev[0]));
        if (hipEventCreate(&ev[1]) != hipSuccess) {
            (void)hipEventDestroy(ev[0]);
            fail(SV_ERR_HIP, "hipEventCreate failed");
        }
        auto timed = [&](int t, bool xcd) {
            SV_HIP(hipEventRecord(ev[0], s->stream));
            launch_half_identity(all_rows(s), t, xcd, s->stream);
            SV_HIP(hipEventRecord(ev[1], s->stream));
            SV_HIP(hipEventSynchronize(ev[1]));
            float ms = 0.0f;
            SV_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            return ms;
        };
        try {
            for (int t = 0; t < n; ++t) {
                if (!half_sweep_applies(n, t)) continue;
                // one untimed sweep per order, then three timed sweeps per
                // order taken alternately; the medians decide
                (void)timed(t, false);
                (void)timed(t, true);
                float a[3], b[3];
                for (int r = 0; r < 3; ++r) {
                    a[r] = timed(t, false);
                    b[r] = timed(t, true);
                }
                std::sort(a, a + 3);
                std::sort(b, b + 3);
                if (b[1] < a[1]) mask |= 1ull << t;
                else mask &= ~(1ull << t);
                if (ms_out) {
                    ms_out[2 * t] = a[1];
                    ms_out[2 * t + 1] = b[1];
                }
            }
        } catch (...) {
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
            throw;
        }
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        set_half_order_mask(n, mask);
    });
}

sv_status sv_sweep_order_set(sv_state s, uint64_t xcd_mask)
{
    return guarded([&] {
        check_state(s);
        set_half_order_mask(s->n, xcd_mask);
    });
}

sv_status sv_sweep_order_get(sv_state s, uint64_t* xcd_mask)
{
    return guarded([&] {
        check_state(s);
        need(xcd_mask != nullptr, SV_ERR_INVALID_ARGUMENT, "xcd_mask is NULL");
        *xcd_mask = half_order_mask(s->n);
    });
}

const char* sv_status_string(sv_status st)
{
    // read as an int: callers may pass any value, and a value outside the
    // enumeration must not be loaded as the enum type
    int code = 0;
    std::memcpy(&code, &st, sizeof code);
    switch (code) {
    case SV_OK: return "ok";
    case SV_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SV_ERR_QUBIT_OUT_OF_RANGE: return "qubit out of range";
    case SV_ERR_QUBIT_OVERLAP: return "qubit used twice";
    case SV_ERR_UNSUPPORTED: return "unsupported";
    case SV_ERR_OUT_OF_MEMORY: return "out of memory";
    case SV_ERR_HIP: return "HIP runtime error";
    case SV_ERR_CAPTURE: return "stream is capturing";
    case SV_ERR_NOT_UNITARY: return "matrix not unitary";
    }
    return "unknown status";
}

const char* sv_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
