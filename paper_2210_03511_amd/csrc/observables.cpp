// Ground-state vectors and expectation values (C ABI): the Ritz vector of
// the tridiagonal T-matrix, a second Lanczos pass that accumulates the
// eigenvector from the Lanczos vectors, and O x and <psi|O|psi> for a
// symmetric operator O evaluated with the H.v kernel on O's own pair table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "basis.h"
#include "launch.h"

using namespace symed;

namespace {

// Solve (T - mu) y = r in place for the symmetric tridiagonal T (diagonal
// a[n], off-diagonal b[n-1]): Gaussian elimination with partial pivoting
// (row interchanges create a second super-diagonal), then back substitution.
// A zero pivot is replaced by a tiny one, as inverse iteration wants the
// nearly singular solve.
void tridiag_solve(const double *a, const double *b, int n, double mu, std::vector<double> &r)
{
    std::vector<double> d(n), du(n, 0.0), du2(n, 0.0), dl(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = a[i] - mu;
    for (int i = 0; i + 1 < n; ++i) du[i] = dl[i] = b[i];
    const double tiny = 1e-300;
    for (int i = 0; i + 1 < n; ++i) {
        if (std::fabs(d[i]) >= std::fabs(dl[i])) {
            if (d[i] == 0.0) d[i] = tiny;
            const double m = dl[i] / d[i];
            d[i + 1] -= m * du[i];
            r[i + 1] -= m * r[i];
        } else {
            // rows i and i+1 exchanged
            const double m = d[i] / dl[i];
            d[i] = dl[i];
            const double t = du[i];
            du[i] = d[i + 1];
            d[i + 1] = t - m * d[i + 1];
            if (i + 2 < n) {
                du2[i] = du[i + 1];
                du[i + 1] = -m * du[i + 1];
            }
            std::swap(r[i], r[i + 1]);
            r[i + 1] -= m * r[i];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = r[i];
        if (i + 1 < n) s -= du[i] * r[i + 1];
        if (i + 2 < n) s -= du2[i] * r[i + 2];
        r[i] = s / (d[i] != 0.0 ? d[i] : tiny);
    }
}

}  // namespace

extern "C" {

ed_status ed_ritz_vector(const double *alpha, const double *beta, int32_t n, int32_t k, double *lambda,
                         double *coef)
{
    if (!alpha || !coef || n < 1 || k < 0 || k >= n || (n > 1 && !beta))
        return fail(ED_EINVAL, "bad arguments");
    std::vector<double> ev(k + 1);
    ed_status st = ed_eigenvalues(alpha, beta, n, k + 1, ev.data());
    if (st != ED_OK) return st;
    const double lam = ev[k];
    if (lambda) *lambda = lam;
    double scale = 0.0;
    for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(alpha[i]));
    for (int i = 0; i + 1 < n; ++i) scale = std::max(scale, std::fabs(beta[i]));
    const double mu = lam + 1e-13 * std::max(scale, 1.0);
    // inverse iteration from a fixed, generic start vector
    std::vector<double> r(n);
    for (int i = 0; i < n; ++i) r[i] = 1.0 + 0.5 * std::sin(1.0 + i);
    for (int it = 0; it < 4; ++it) {
        tridiag_solve(alpha, beta, n, mu, r);
        double nr = 0.0;
        for (double x : r) nr += x * x;
        nr = std::sqrt(nr);
        if (!(nr > 0.0) || !std::isfinite(nr)) return fail(ED_EINVAL, "inverse iteration failed");
        for (double &x : r) x /= nr;
    }
    // sign convention: first non-negligible coefficient positive
    for (int i = 0; i < n; ++i)
        if (std::fabs(r[i]) > 1e-8) {
            if (r[i] < 0)
                for (double &x : r) x = -x;
            break;
        }
    std::copy(r.begin(), r.end(), coef);
    return ED_OK;
}

ed_status ed_lanczos_vector(const ed_basis *cb, const void *d_v0, int32_t n_iter, int32_t lookup_mode,
                            const double *h_coef, void *d_psi, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(cb);
    if (!b || !d_v0 || !h_coef || !d_psi) return fail(ED_EINVAL, "bad arguments");
    if (d_psi == d_v0) return fail(ED_EINVAL, "psi must not alias v0");
    b->lanczos_steps = -1;  // the second pass replaces the run's state
    ed_status st = lanczos_prepare(b, n_iter, lookup_mode, 0);
    if (st != ED_OK) return st;
    const bool cplx = b->T.is_complex;
    const int64_t n2 = b->dim * (cplx ? 2 : 1);
    double *d_coef = nullptr;
    TmpPool tmp(b);
    if ((st = tmp.take((void **)&d_coef, n_iter * sizeof(double))) != ED_OK) return st;
    hipStream_t s = b->own;
    auto done = [&](ed_status r) {
        (void)hipStreamSynchronize(s);  // before the pool frees the coefficients
        return r;
    };
    if ((st = lanczos_start(b, d_v0, stream)) != ED_OK) return done(st);
    // the same steps again; before step k, psi += coef[k] v_k
    hipError_t e = hipMemcpyAsync(d_coef, h_coef, n_iter * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill(static_cast<double *>(d_psi), n2, 0.0, b->cfg.vec_blocks, s);
    for (int k = 0; k < n_iter && e == hipSuccess; ++k) {
        e = launch_axpy_coef(static_cast<double *>(d_psi), b->d_v, n2, d_coef, b->d_ls, b->cfg.vec_blocks, s);
        if (e == hipSuccess) e = hipGraphLaunch(b->step_graph[lookup_mode], s);
    }
    // normalize psi
    if (e == hipSuccess) e = launch_norm2_partial(d_psi, b->dim, cplx, b->d_partials, b->cfg.vec_blocks, s);
    if (e == hipSuccess)
        e = launch_scale_copy(d_psi, d_psi, b->dim, cplx, b->d_partials, b->cfg.vec_blocks, b->cfg.vec_blocks, s);
    if (e != hipSuccess) return done(fail(ED_EDEVICE, std::string("second Lanczos pass: ") + hipGetErrorString(e)));
    return done(ED_OK);
}

}  // extern "C"

namespace {

// Tables of an operator O of the same form as H (bonds, chirality
// triangles), which must be invariant under the basis's group: O's pair
// table in place of H's, in a blob laid out like the basis's (lay2).  The
// learned index network, which lives in the blob, is carried over by
// op_apply.  Host only.
ed_status op_tables(const ed_basis *b, const ed_model *op, int32_t lookup_mode, std::vector<uint8_t> &blob,
                    BlobLayout &lay2, int &n_pairs)
{
    if (b->T.n_colors) return fail(ED_EINVAL, "spin-1/2 operators do not act on an SU(d) basis");
    if (!(lookup_mode == 0 || (lookup_mode == 1 && b->indexed) || (lookup_mode == 2 && b->hashed)))
        return fail(ED_EINVAL, "lookup_mode not available on this basis");
    if (op->n_sites != b->T.N) return fail(ED_EINVAL, "operator on another number of sites");
    if ((op->n_bonds > 0 && (!op->bond_sites || !op->bond_J)) || (op->n_tri > 0 && (!op->tri_sites || !op->tri_Jchi)) ||
        op->n_bonds < 0 || op->n_tri < 0)
        return fail(ED_EINVAL, "operator arrays");
    for (int q = 0; q < 2 * op->n_bonds; ++q)
        if (op->bond_sites[q] < 0 || op->bond_sites[q] >= op->n_sites) return fail(ED_EINVAL, "bond site out of range");
    for (int q = 0; q < 2 * op->n_bonds; q += 2)
        if (op->bond_sites[q] == op->bond_sites[q + 1]) return fail(ED_EINVAL, "bond on one site");
    for (int q = 0; q < 3 * op->n_tri; ++q)
        if (op->tri_sites[q] < 0 || op->tri_sites[q] >= op->n_sites) return fail(ED_EINVAL, "triangle site out of range");
    bool chir = false;
    for (int t = 0; t < op->n_tri; ++t) chir |= op->tri_Jchi[t] != 0.0;
    if (chir && !b->T.is_complex) return fail(ED_EINVAL, "a chirality operator needs a complex sector");
    HostTables T2 = b->T;
    ed_status st = check_invariant(op, T2);
    if (st != ED_OK) return st;
    build_pairs(op, T2);
    lay2 = BlobLayout{};
    blob = pack_blob(T2, lay2);
    n_pairs = (int)T2.pairs.size();
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) != hipSuccess)
        return fail(ED_EDEVICE, "device query");
    if ((int64_t)lay2.bytes + (b->lay.bytes - b->lay.off_mlp) + 256 > lds_max)
        return fail(ED_EINVAL, "operator tables exceed the LDS of one block");
    // the learned index's network pieces and rank table are copied in behind
    // the tables, at the same offsets relative to off_mlp
    if (b->indexed) {
        lay2.off_rank = lay2.off_mlp + (b->lay.off_rank - b->lay.off_mlp);
        lay2.bytes = lay2.off_mlp + (b->lay.bytes - b->lay.off_mlp);
    }
    return ED_OK;
}

// Bytes of device memory an operator blob takes (tables, and the carried
// network pieces).
size_t op_blob_bytes(const ed_basis *b, const std::vector<uint8_t> &blob, const BlobLayout &lay2)
{
    size_t n = blob.size();
    if (b->indexed) n = std::max(n, (size_t)lay2.bytes);
    return (n + 255) & ~(size_t)255;
}

// y = O x, enqueued on s with O's blob copied to d_blob (op_blob_bytes of
// device memory); the caller synchronizes before the host blob or d_blob go.
ed_status op_apply(ed_basis *b, const std::vector<uint8_t> &blob, const BlobLayout &lay2, int n_pairs, void *d_blob,
                   const void *d_x, void *d_y, int32_t lookup_mode, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(d_blob, blob.data(), blob.size(), hipMemcpyHostToDevice, s);
    // the learned index's network and rank table live in the blob: carry them over
    if (e == hipSuccess && b->indexed)
        e = hipMemcpyAsync(static_cast<unsigned char *>(d_blob) + lay2.off_mlp,
                           static_cast<const unsigned char *>(b->d_blob) + b->lay.off_mlp,
                           b->lay.bytes - b->lay.off_mlp, hipMemcpyDeviceToDevice, s);
    KParams p = make_params(b);
    p.lay = lay2;
    p.blob = d_blob;
    p.n_pairs = n_pairs;
    int bpc = 0, thr = 0;
    if (e == hipSuccess) e = prepare_kernels(p, &bpc, &thr);
    if (e == hipSuccess) e = stage_input(b, lookup_mode, d_x, s);
    if (e == hipSuccess) e = launch_apply(p, b->cfg, d_x, d_y, 0, lookup_mode, nullptr, nullptr, s);
    if (e != hipSuccess) return fail(ED_EDEVICE, std::string("operator apply: ") + hipGetErrorString(e));
    return ED_OK;
}

// <z, y> = sum conj(z_i) y_i from the per-block partials of the dot kernel
// (d_part: 2 * vec_blocks doubles); synchronizes s.
ed_status op_dot(ed_basis *b, const void *d_z, const void *d_y, double *d_part, double *h_re, double *h_im,
                 hipStream_t s)
{
    const bool cplx = b->T.is_complex;
    const int nb = b->cfg.vec_blocks;
    std::vector<double> part(2 * nb, 0.0);
    hipError_t e = launch_dot(d_z, d_y, b->dim, cplx, d_part, nb, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(part.data(), d_part, (cplx ? 2 : 1) * nb * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(ED_EDEVICE, std::string("dot product: ") + hipGetErrorString(e));
    double re = 0.0, im = 0.0;
    for (int q = 0; q < nb; ++q) re += part[q];
    if (cplx)
        for (int q = 0; q < nb; ++q) im += part[nb + q];
    *h_re = re;
    if (h_im) *h_im = im;
    return ED_OK;
}

// Scratch memory of ed_apply_op_noalloc: the operator's table blob, then
// the dot partials, on every device the library runs on (each holds its own
// copy until the process ends).  Host code never uses the array's name as an
// address: the device address of each device's copy comes from
// hipGetSymbolAddress at the first call on that device.
constexpr size_t kScratchBytes = 256u << 10;
constexpr size_t kScratchPartials = 32u << 10;     // dot partials at the end
constexpr size_t kScratchBlob = kScratchBytes - kScratchPartials;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
static ed_status scratch_address(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(ED_EINVAL, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ED_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[device]);
    return ED_OK;
}

}  // namespace

extern "C" {

ed_status ed_apply_op(const ed_basis *cb, const ed_model *op, const void *d_x, void *d_y, const void *d_z,
                      int32_t lookup_mode, double *h_re, double *h_im, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(cb);
    if (!b || !op || !d_x || !d_y || (d_z && !h_re)) return fail(ED_EINVAL, "bad arguments");
    if (d_x == d_y) return fail(ED_EINVAL, "y must not alias x");
    if (d_z) {
        *h_re = 0.0;
        if (h_im) *h_im = 0.0;
    }
    if (b->dim == 0) return ED_OK;
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint8_t> blob;
    BlobLayout lay2{};
    int n_pairs = 0;
    ed_status st = op_tables(b, op, lookup_mode, blob, lay2, n_pairs);
    if (st != ED_OK) return st;
    TmpPool tmp(b);
    void *d_blob = nullptr;
    double *d_part = nullptr;
    if ((st = tmp.take(&d_blob, op_blob_bytes(b, blob, lay2))) != ED_OK) return st;
    if (d_z && (st = tmp.take((void **)&d_part, 2 * b->cfg.vec_blocks * sizeof(double))) != ED_OK) return st;
    st = op_apply(b, blob, lay2, n_pairs, d_blob, d_x, d_y, lookup_mode, s);
    if (st == ED_OK && d_z) st = op_dot(b, d_z, d_y, d_part, h_re, h_im, s);
    (void)hipStreamSynchronize(s);  // before the pool and the host blob go
    return st;
}

ed_status ed_expectation(const ed_basis *cb, const ed_model *op, const void *d_psi, int32_t lookup_mode,
                         double *h_re, double *h_im, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(cb);
    if (!b || !op || !d_psi || !h_re) return fail(ED_EINVAL, "bad arguments");
    if (b->dim == 0) {
        *h_re = 0.0;
        if (h_im) *h_im = 0.0;
        return ED_OK;
    }
    const bool cplx = b->T.is_complex;
    const size_t vbytes = (size_t)b->dim * sizeof(double) * (cplx ? 2 : 1);
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint8_t> blob;
    BlobLayout lay2{};
    int n_pairs = 0;
    ed_status st = op_tables(b, op, lookup_mode, blob, lay2, n_pairs);
    if (st != ED_OK) return st;
    TmpPool tmp(b);
    void *d_blob = nullptr, *d_y = nullptr;
    double *d_part = nullptr;
    if ((st = tmp.take(&d_y, vbytes)) != ED_OK) return st;
    if ((st = tmp.take((void **)&d_part, 2 * b->cfg.vec_blocks * sizeof(double))) != ED_OK) return st;
    if ((st = tmp.take(&d_blob, op_blob_bytes(b, blob, lay2))) != ED_OK) return st;
    st = op_apply(b, blob, lay2, n_pairs, d_blob, d_psi, d_y, lookup_mode, s);
    if (st == ED_OK) st = op_dot(b, d_psi, d_y, d_part, h_re, h_im, s);
    (void)hipStreamSynchronize(s);
    return st;
}

ed_status ed_apply_op_noalloc(const ed_basis *cb, const ed_model *op, const void *d_x, void *d_y, const void *d_z,
                              int32_t lookup_mode, double *h_re, double *h_im, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(cb);
    if (!b || !op || !d_x || !d_y || (d_z && !h_re)) return fail(ED_EINVAL, "bad arguments");
    if (d_x == d_y) return fail(ED_EINVAL, "y must not alias x");
    if (d_z) {
        *h_re = 0.0;
        if (h_im) *h_im = 0.0;
    }
    if (b->dim == 0) return ED_OK;
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint8_t> blob;
    BlobLayout lay2{};
    int n_pairs = 0;
    ed_status st = op_tables(b, op, lookup_mode, blob, lay2, n_pairs);
    if (st != ED_OK) return st;
    const size_t need = op_blob_bytes(b, blob, lay2);
    if (need > kScratchBlob)
        return fail(ED_EINVAL, "operator tables (" + std::to_string(need) + " B) exceed the scratch space of " +
                                   std::to_string(kScratchBlob) + " B");
    if (d_z && 2 * (size_t)b->cfg.vec_blocks * sizeof(double) > kScratchPartials)
        return fail(ED_EINVAL, "dot partials exceed the scratch space of " + std::to_string(kScratchPartials) + " B");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ED_EDEVICE, "hipGetDevice");
    if (dev != b->device) return fail(ED_EINVAL, "the basis lives on another device than the current one");
    unsigned char *base = nullptr;
    if ((st = scratch_address(dev, &base)) != ED_OK) return st;
    st = op_apply(b, blob, lay2, n_pairs, base, d_x, d_y, lookup_mode, s);
    if (st == ED_OK && d_z)
        st = op_dot(b, d_z, d_y, reinterpret_cast<double *>(base + kScratchBlob), h_re, h_im, s);
    (void)hipStreamSynchronize(s);  // before the host blob goes
    return st;
}

}  // extern "C"
