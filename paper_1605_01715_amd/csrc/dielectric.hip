// The dielectric problem around the solve (Sec. II.C): the right-hand side
// with free charges (Eqs. rhs, Ef) and the forces on the bodies.
//
// Both need the field of a surface charge at the surface points: the
// single-layer field output of the plan (the sum over k != j of
// (r_j - r_k) s_k a_k / (4 pi r^3)) plus the self-patch term of Eq.
// pol_discret, read as s_j sqrt(pi a_j) H_j / (4 pi) along n_j (the
// principal-value field of a uniformly charged spherical cap of area a_j).
#include <cmath>
#include <mutex>

#include "plan.hpp"

namespace fmm {

namespace {

constexpr int kBlock = 256;
constexpr float kInv4PiF = 0.079577471545947667884f;

__global__ void k_charge(const float *sigma, const float *sigma2, const float *areas, float *dens, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float s = sigma[i] + (sigma2 ? sigma2[i] : 0.f);
    dens[i] = s * areas[i];
}

// total field at element i: plan field + self term along n + E0
__device__ inline void total_field(int64_t i, const float *field, const float *nrm, const float *sigma,
                                   const float *sigma2, const float *areas, const float *curv, double e0x, double e0y,
                                   double e0z, double *e, double *nv) {
    const double s = (double)sigma[i] + (sigma2 ? (double)sigma2[i] : 0.0);
    const double self = s * std::sqrt(3.14159265358979323846 * (double)areas[i]) * (double)curv[i] * (double)kInv4PiF;
    for (int c = 0; c < 3; ++c) nv[c] = nrm[3 * i + c];
    e[0] = field[3 * i] + self * nv[0] + e0x;
    e[1] = field[3 * i + 1] + self * nv[1] + e0y;
    e[2] = field[3 * i + 2] + self * nv[2] + e0z;
}

// b = (1 - ebar) sigma_f - deps n . E,  ebar = (eps_i + eps_m)/2, deps = eps_m - eps_i
__global__ void k_rhs(const float *field, const float *nrm, const float *sf, const float *areas, const float *curv,
                      const float *eps_i, double eps_m, double e0x, double e0y, double e0z, double *b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double e[3], nv[3];
    total_field(i, field, nrm, sf, nullptr, areas, curv, e0x, e0y, e0z, e, nv);
    const double ei = eps_i[i];
    const double ebar = 0.5 * (ei + eps_m), deps = eps_m - ei;
    b[i] = (1.0 - ebar) * (double)sf[i] - deps * (e[0] * nv[0] + e[1] * nv[1] + e[2] * nv[2]);
}

// per-body force: one block per body sums eps_m s a E over its elements in a
// fixed order (deterministic)
__global__ __launch_bounds__(kBlock) void k_body_force(const float *field, const float *nrm, const float *sigma,
                                                       const float *sigma2, const float *areas, const float *curv,
                                                       double eps_m, double e0x, double e0y, double e0z,
                                                       const int64_t *off, double *out) {
    __shared__ double sh[3][kBlock];
    const int b = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += kBlock) {
        double e[3], nv[3];
        total_field(i, field, nrm, sigma, sigma2, areas, curv, e0x, e0y, e0z, e, nv);
        const double w = eps_m * ((double)sigma[i] + (sigma2 ? (double)sigma2[i] : 0.0)) * (double)areas[i];
        for (int c = 0; c < 3; ++c) acc[c] += w * e[c];
    }
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) out[3 * b + c] = sh[c][0];
}

void require_field_plan(const Plan &P, const char *who) {
    FMM_REQUIRE(P.sl && P.want_field, std::string(who) + ": needs a single-layer plan with field output");
    FMM_REQUIRE(!P.t.tsm, std::string(who) + ": targets must be the sources");
    FMM_REQUIRE(P.nrhs == 1, std::string(who) + ": the plan must have nrhs = 1");
    FMM_REQUIRE(P.trg_nrm_user.n > 0, std::string(who) + ": the plan needs target normals");
}

// field of the charge (sigma + sigma2) * areas, caller's order, [n][3], into
// dens [n] (the charge) and field [3 n]; stream-ordered
void charge_field_into(Plan &P, const float *sigma, const float *sigma2, const float *areas, float *dens, float *field,
                       hipStream_t s) {
    const int64_t n = P.t.n_src;
    hipLaunchKernelGGL(k_charge, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, sigma, sigma2, areas, dens, n);
    FMM_HIP(hipGetLastError());
    plan_apply(P, dens, nullptr, nullptr, field, s);
}

void charge_field(Plan &P, const float *sigma, const float *sigma2, const float *areas, DBuf<float> &field,
                  hipStream_t s) {
    const int64_t n = P.t.n_src;
    DBuf<float> dens(n);
    field.alloc(3 * n);
    charge_field_into(P, sigma, sigma2, areas, dens.p, field.p, s);
    FMM_HIP(hipStreamSynchronize(s));  // dens is freed on return
}

void launch_rhs(const Plan &P, const float *field, const float *sigma_f, const float *areas, const float *curv,
                const float *eps_i, double eps_m, const double *e0, double *b, hipStream_t s) {
    const int64_t n = P.t.n_src;
    const double ex = e0 ? e0[0] : 0.0, ey = e0 ? e0[1] : 0.0, ez = e0 ? e0[2] : 0.0;
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, field, P.trg_nrm_user.p, sigma_f, areas,
                       curv, eps_i, eps_m, ex, ey, ez, b, n);
    FMM_HIP(hipGetLastError());
}

}  // namespace

void dielectric_rhs(Plan &P, const float *sigma_f, const float *areas, const float *curv, const float *eps_i,
                    double eps_m, const double *e0, double *b, hipStream_t s) {
    require_field_plan(P, "fmm_dielectric_rhs");
    const int64_t n = P.t.n_src;
    if (n == 0) return;
    DBuf<float> field;
    charge_field(P, sigma_f, nullptr, areas, field, s);
    launch_rhs(P, field.p, sigma_f, areas, curv, eps_i, eps_m, e0, b, s);
    FMM_HIP(hipStreamSynchronize(s));
}

// Scratch of dielectric_rhs_noalloc, one copy per GPU for the life of the
// process: the charge density (n floats) and its field (3 n floats, from a
// 256-byte boundary) of the last call on that GPU. Calls that overlap in time
// on one GPU race on it. Nothing in it needs clearing: both parts are fully
// written before they are read.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current. The array's own name is a host-side stand-in and
// is never passed to a kernel or a copy.
unsigned char *scratch_address() {
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    FMM_REQUIRE(dev >= 0 && dev < kMaxDevices, "scratch: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        FMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        FMM_REQUIRE(p != nullptr, "scratch: no device address");
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[dev]);
}

}  // namespace

void dielectric_rhs_noalloc(Plan &P, const float *sigma_f, const float *areas, const float *curv,
                            const float *eps_i, double eps_m, const double *e0, double *b, hipStream_t s) {
    require_field_plan(P, "fmm_dielectric_rhs_noalloc");
    const int64_t n = P.t.n_src;
    FMM_REQUIRE(n <= kNoAllocMaxPoints, "fmm_dielectric_rhs_noalloc: more points than the fixed scratch holds (" +
                                            std::to_string(kNoAllocMaxPoints) + ")");
    if (n == 0) return;
    const size_t field_off = ((size_t)n * sizeof(float) + 255) / 256 * 256;
    static_assert(((size_t)kNoAllocMaxPoints * 4 + 255) / 256 * 256 + (size_t)kNoAllocMaxPoints * 12 <=
                      kNoAllocScratchBytes,
                  "scratch too small for the point limit");
    unsigned char *base = scratch_address();
    float *dens = reinterpret_cast<float *>(base);
    float *field = reinterpret_cast<float *>(base + field_off);
    charge_field_into(P, sigma_f, nullptr, areas, dens, field, s);
    launch_rhs(P, field, sigma_f, areas, curv, eps_i, eps_m, e0, b, s);
}

void body_forces(Plan &P, const float *sigma, const float *sigma2, const float *areas, const float *curv,
                 double eps_m, const double *e0, int n_body, const int64_t *body_off, double *forces, hipStream_t s) {
    require_field_plan(P, "fmm_body_forces");
    const int64_t n = P.t.n_src;
    FMM_REQUIRE(n_body >= 1 && body_off, "fmm_body_forces: need n_body >= 1 and body offsets");
    FMM_REQUIRE(body_off[0] == 0 && body_off[n_body] == n, "fmm_body_forces: body offsets must span 0..n");
    for (int i = 0; i < n_body; ++i)
        FMM_REQUIRE(body_off[i + 1] >= body_off[i], "fmm_body_forces: body offsets must be nondecreasing");
    DBuf<float> field;
    if (n) charge_field(P, sigma, sigma2, areas, field, s);
    std::vector<int64_t> off(body_off, body_off + n_body + 1);
    DBuf<int64_t> doff = upload(off, s);
    DBuf<double> out(3 * (size_t)n_body);
    const double ex = e0 ? e0[0] : 0.0, ey = e0 ? e0[1] : 0.0, ez = e0 ? e0[2] : 0.0;
    hipLaunchKernelGGL(k_body_force, dim3(n_body), dim3(kBlock), 0, s, field.p, P.trg_nrm_user.p, sigma, sigma2,
                       areas, curv, eps_m, ex, ey, ez, doff.p, out.p);
    FMM_HIP(hipGetLastError());
    d2h(forces, out.p, 3 * (size_t)n_body, s);
}

}  // namespace fmm
