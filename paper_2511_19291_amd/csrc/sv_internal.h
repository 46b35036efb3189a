// sv_internal.h -- host-side structures and launcher declarations shared by
// the translation units of libsv.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sv.h"

namespace sv {

using cd = std::complex<double>;

// ------------------------------------------------------------ errors

struct Error {
    sv_status st;
    std::string msg;
};

[[noreturn]] void fail(sv_status st, const std::string& msg);
void set_last_error(const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define SV_HIP(call) ::sv::hip_check((call), #call)

// ------------------------------------------------------------ device info

struct DeviceInfo {
    int cu_count = 256;
    int device = 0;
};
const DeviceInfo& device_info();

// ------------------------------------------------------------ gate math (host, complex128)

// Matrix of a named kind at the given parameters; returns k. Row-major,
// first target = most significant bit of the index.
int kind_matrix(int kind, const double* prm, cd* m);
// d M / d prm[j]; returns k or -1 if the kind has no parameter j.
int kind_dmatrix(int kind, const double* prm, int j, cd* m);
int kind_targets(int kind);
int kind_nparams(int kind);
// Matrix of a circuit op (named kind at its parameters, or its explicit
// matrix); *k = number of targets.
void gate_matrix_of_op(const sv_op& op, const double* params, cd* m, int* k);

// ------------------------------------------------------------ kernel launch arguments

// Row addressing: rows [0, nrow0) start at p0 + r * N, rows [nrow0, nrows)
// at p1 + (r - nrow0) * N. Lets one launch sweep psi and lambda together.
struct Rows {
    float2* p0;
    float2* p1;
    int nrow0;
    int nrows;
    uint64_t N;
};

struct GateLaunch {
    Rows rows;
    int k;                    // 1 or 2 targets
    int targets[2];
    int nc;
    int controls[SV_MAX_CONTROLS];
    float2 m[16];             // complex64 matrix (k=1 uses 4)
};

struct DiagLaunch {
    Rows rows;
    int nfixed;               // qubits fixed to 1 (controls, and targets in "ones" mode)
    int fixed[SV_MAX_CONTROLS + 2];
    int nfree;                // targets whose bit selects the phase
    int freeq[2];
    float2 ph[4];             // phase per free-target bit pattern (free[0] = MSB)
};

// Plain gate kernels (k_gates.hip). All asynchronous on `st`.
void launch_gate(const GateLaunch& g, hipStream_t st);
// Workgroup order of the uncontrolled split-halves sweep (one target >= 7,
// states of >= 8 qubits), per device and state size: bit t of the mask set =
// XCD-contiguous order on target t, clear = the hardware's order (default).
uint64_t half_order_mask(int n);
void set_half_order_mask(int n, uint64_t mask);
bool half_sweep_applies(int n, int t);
// One split-halves sweep of the identity on target t in the given order (the
// values are unchanged: x*1 + y*0); for timing the two orders.
void launch_half_identity(const Rows& rows, int t, bool xcd, hipStream_t st);
void launch_diag(const DiagLaunch& d, hipStream_t st);
void launch_basis(const Rows& r, uint64_t idx, hipStream_t st);
void launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t st);

// Reductions (k_reduce.hip). Partial buffers are device memory owned by the
// caller; sizes from the *_parts functions.
uint64_t zall_parts(int n, int rows);                 // doubles of scratch
void launch_zall(const Rows& r, int n, double* scratch, double* out /*[rows][n+1]*/, hipStream_t st);
// Size (doubles) of the library's fixed device buffer for the allocation-free
// <Z_i> reduction, and its address on the current device (looked up once per
// device with hipGetSymbolAddress).
constexpr uint64_t kStaticZallDoubles = 1ull << 20;   // 8 MiB
double* static_zall_scratch();

struct PauliGroup {             // terms sharing one x mask
    uint64_t x_mask;
    int nt;
    uint64_t z_mask[8];
    int y_count[8];             // popcount(x & z) per term
};
uint64_t pauli_parts(int n, int rows, int nt);
void launch_pauli_group(const Rows& r, int n, const PauliGroup& g, double* scratch,
                        double* out /*[rows][nt]*/, hipStream_t st);

// inner: out[2r] = Re sum conj(a) b, out[2r + 1] = Im (FP64).
uint64_t inner_parts(int n, int rows);
void launch_inner(const Rows& a, const Rows& b, int n, double* scratch, double* out, hipStream_t st);
// out[r] = || psi_r - e_0 ||^2
uint64_t drift_parts(int n, int rows);
void launch_drift(const Rows& a, int n, double* scratch, double* out, hipStream_t st);

// Adjoint (k_adjoint.hip).
struct PauliTermDev {
    uint64_t x_mask, z_mask;
    double coeff;
    int y_count;
    int orig;                 // index of the term in the caller's list
};
// lam <- O psi, O = sum of terms (device array of nt terms). coeff_rows:
// NULL, or device [rows][nt] coefficients (caller's term order) replacing
// each term's coeff row by row. zonly: every term is a single-qubit Z (the
// table path).
void launch_diag_lambda(const Rows& psi, const Rows& lam, int n, const double* w, hipStream_t st);
void launch_apply_pauli_sum(const Rows& psi, const Rows& lam, int n, const PauliTermDev* terms, int nt,
                            const double* coeff_rows, hipStream_t st,
                            bool zonly = false);

// ------------------------------------------------------------ shots
struct ShotLaunch {
    const float2* psi;        // one row of 2^n amplitudes
    int n;
    const double* u;          // device uniforms [shots]
    int64_t shots;
    int64_t* out;             // device indices [shots]
    void* scratch;            // shot_scratch_bytes(n, shots) bytes
};
size_t shot_scratch_bytes(int n, int64_t shots);
void launch_sample_exact(const ShotLaunch& a, hipStream_t st);

// <Z_i> estimates from n_shots drawn indices (-1 = no index): est[n] device
// doubles; scratch holds n + 1 counters (8 bytes each).
void launch_shot_zest(const int64_t* idx, int64_t shots, int n, void* scratch, double* est, hipStream_t st);

struct GaussLaunch {
    const float2* psi;        // one row
    int n;
    const double* z;          // device normals [2^n]
    double shots;
    double* y;                // device output [2^n]
    double* scratch;          // gauss_scratch_doubles(n) doubles
};
uint64_t gauss_scratch_doubles(int n);
void launch_sample_gaussian(const GaussLaunch& a, hipStream_t st);

// Gaussian estimate of every <Z_i> (E_i = (1/shots) sum_b y_b s_i(b)) and
// its backward: w_b = dF/d|psi_b|^2 for F = sum_i g_i E_i, normals fixed.
struct GaussZLaunch {
    const float2* psi;        // one row
    int n;
    const double* z;          // device normals [2^n]
    double shots;
    double g[SV_MAX_QUBITS];  // upstream dF/dE_i (backward)
    double* est;              // device [n] (forward)
    double* w;                // device [2^n] (backward)
    double* scratch;          // gauss_z_scratch_doubles(n) doubles
};
uint64_t gauss_z_scratch_doubles(int n);
void launch_gauss_z(const GaussZLaunch& a, hipStream_t st);
void launch_gauss_z_backward(const GaussZLaunch& a, hipStream_t st);

// ------------------------------------------------------ matrix-core adjoint
// One sweep per block of gates on four qubits: the block's correlation
// S = sum_c psi_c lambda_c^* (as S_real, 32 x 32 FP64 per row) and the
// un-apply of the block's product from psi and lambda.
struct AdjMfmaLaunch {
    Rows psi;
    Rows lam;
    uint64_t N;
    int q[4];                 // block qubits, ascending
    const float* frag;        // 64 lanes x 16 floats: operands of [[Re M, -Im M], [Im M, Re M]], M = U_B^*
    int frag_stride;          // floats between rows' operands (0: one product for all rows)
    double* spart;            // adj_mfma_part_doubles(grid, rows): [rows][grid][kAmPart], then the level sums
    int grid;                 // workgroups per row
    int gpw;                  // groups (of 512 amplitudes) per wave
};
constexpr int kAmPart = 512;                   // doubles of a workgroup's part: Re S, Im S (16 x 16 each)
constexpr int kAmMinGpw = 4;                   // default groups per wave
constexpr uint64_t kAmMaxParts = 1ull << 16;   // workgroups of one launch, all rows
struct AdjMfmaShape {
    int grid;                 // workgroups per row
    int gpw;                  // groups per wave
};
AdjMfmaShape adj_mfma_shape(int n, int rows, int min_gpw = kAmMinGpw);
uint64_t adj_mfma_part_doubles(int grid, int rows);
void launch_adj_mfma(const AdjMfmaLaunch& a, int rows, double* s_out, hipStream_t st);

// ------------------------------------------------------------ blocked adjoint
// Block planning on qubit masks only (the fusion planners): per block its
// qubits and its gates (indices into the mask list, circuit order).
struct GateBlock {
    std::vector<int> qs;
    std::vector<int> gates;
};
std::vector<GateBlock> plan_gate_blocks(const std::vector<uint64_t>& masks, int max_k);

constexpr int kAdjBlockMaxBits = 5;       // local bits of a column (8, 16 or 32 amplitudes)
constexpr int kAdjBlockMaxSlots = 64;     // derivative slots per block launch

// One gate of a block, in local bit positions.
struct AdjBlockGate {
    int nt;                   // 1 or 2 targets
    int t0, t1;               // local target bits (t0 = most significant matrix bit)
    int cmask;                // local control bits
    int nd;                   // derivatives (0..3; at most 1 for two targets)
    int slot[3];              // slot of each derivative within the launch
    int form;                 // U^*: 0 dense, 1 diagonal, 2 plain exchange (X)
    int pauli;                // derivative of exp(-i theta P / 2): 1 X, 2 Y, 3 Z, 4 XX, 5 YY, 6 ZZ; 0 general
    float2 u[16];             // U^* (complex64)
    double2 g[3][16];         // G_d = dU/dtheta_d U^* (complex128), general derivatives
};

struct AdjBlockLaunch {
    Rows psi;
    Rows lam;
    uint64_t qbit[kAdjBlockMaxBits]; // 1 << qubit of each local bit (ascending qubits)
    int q[kAdjBlockMaxBits];
    int lb;                          // local bits: 3, 4 or 5
    int ngates;
    const AdjBlockGate* gates;       // device, in un-apply order (the block's last gate first)
    int nslots;
    int grid;                        // workgroups per row
};
// partials: part[(row * nslots + s) * (4 * grid) + wave]
void launch_adj_block(const AdjBlockLaunch& a, double* part, hipStream_t st);
int adj_block_grid(int n, int lb);

struct AdjLaunch {
    Rows psi;                 // rows of psi
    Rows lam;                 // rows of lambda (same count)
    int k;
    int targets[2];
    int nc;
    int controls[SV_MAX_CONTROLS];
    float2 uinv[16];          // U^* in complex64
    int nd;                   // derivative count (<= 3)
    double2 g[3][16];         // G_j = dU/dtheta_j U^* in complex128
    int grid;                 // blocks per row (the slot stride of the partials)
};
int adj_grid(int n, int k, int nc);                   // blocks per row for a gate's unit count
// partial sums land in part[(row * nd + j) * grid + block]
void launch_adj_step(const AdjLaunch& a, double* part, hipStream_t st);
// out[s] = sum_b part[s * grid + b], s < nslots
void launch_sum_slots(const double* part, int grid, int nslots, double* out, hipStream_t st);

// Fused blocks (k_fused.hip).
struct FusedLaunch {
    float2* psi;
    uint64_t N;
    int nrows;
    int targets[5];           // exactly five (padded with identity qubits)
    int mode;                 // SV_FUSED_FP32_MFMA or SV_FUSED_BF16X3
    const float* amat;        // device: real 64x64 embedding (FP32) or hi then lo parts (BF16X3), then
                              // the products' left operands in fragment order (FP32 values, or BF16
                              // hi and lo bits); 3 x 4096 floats per matrix
    uint32_t amat_stride;     // floats between batch rows' matrices (0: one matrix for every row)
};
void launch_fused_mfma(const FusedLaunch& f, hipStream_t st);

// Six-qubit blocks (BF16x3, all targets >= 6, 12 <= n <= 32).
struct Fused6Launch {
    float2* psi;
    uint64_t N;
    int nrows;
    int targets[6];
    const uint16_t* amat;     // device: fused6_matrix_bytes() in the kernel's layout
};
size_t fused6_matrix_bytes();
// BF16 hi / lo parts of the real 128 x 128 embedding (row-major floats
// holding BF16 values) -> the kernel's padded layout.
void fused6_layout(const float* embed_hi, const float* embed_lo, uint16_t* out);
void launch_fused_wide6(const Fused6Launch& f, hipStream_t st);

struct FusedValuLaunch {
    float2* psi;
    uint64_t N;
    int nrows;
    int k;
    const int* pos;           // device: sorted target positions (k entries)
    const uint64_t* moff;     // device: member offsets (2^k entries)
    const float2* m;          // device: 2^k x 2^k complex64
};
void launch_fused_valu(const FusedValuLaunch& f, hipStream_t st);

}  // namespace sv

// sv_state handle
struct sv_state_s {
    int n = 0;
    int batch = 0;
    uint64_t N = 0;
    float2* psi = nullptr;
    bool owns = false;
    hipStream_t stream = nullptr;
    float2* lam = nullptr;          // adjoint buffer (owned)
    double* scratch = nullptr;      // device reduction scratch
    size_t scratch_cap = 0;         // doubles
    double* dout = nullptr;         // device small outputs
    size_t dout_cap = 0;            // doubles
    double* hout = nullptr;         // pinned host mirror of dout
    float* hstage = nullptr;        // pinned host staging for uploads
    size_t hstage_cap = 0;          // floats
    hipEvent_t events[16] = {};     // completion marks of a call's chunks (created on first use)
    void* dterms = nullptr;         // device copy of observable terms
    size_t dterms_cap = 0;
    void* dfused = nullptr;         // device copy of fused block matrices
    size_t dfused_cap = 0;
    bool failed = false;            // a HIP call failed during a call on this state (sticky)
    std::string failed_msg;         // that failure's detail
    bool inject_hip_error = false;  // testing hook: fail the next call as a HIP error
};
