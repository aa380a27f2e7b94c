// Closure network object (mlb_net): parameters, buffers and the training
// step of the force-closure CNN, on the caller's workspace.
//
// Parameters cross the ABI in float32 in the order layer by layer, weights
// W[co][ci][kz][ky][kx] then biases b[co]; on the device each layer keeps a
// float32 master copy, the Adam moments and bfloat16 copies in the
// kernels' layouts [tap][co][ci] (forward) and [tap][ci][co] (data
// gradient), padded to the kernels' channel counts with zeros.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlb.h"
#include "cnn.h"
#include "net_internal.h"

struct mlb_net_s {
    int nx = 0, ny = 0, nz = 0, training = 0;
    long long N = 0;
    char *ws = nullptr;
    size_t total = 0;
    struct Layer {
        size_t w, m, v, gw, wb, wt, b, mb, vb, gb;
        int nw, cop, cip, cout, cin;
    } L[mlb::kNetLayers];
    size_t x = 0, a[3] = {0, 0, 0}, z[3] = {0, 0, 0}, y = 0, tg = 0, g3 = 0, g[2] = {0, 0};
    size_t part = 0, loss = 0, err = 0, nc = 0, pool = 0;
    int nblk = 0;
    float n_ref = 1.f, j_ref = 1.f, f_ref = 1.f;
    // bumped whenever something a captured inference graph bakes in (the
    // scales, passed as kernel arguments) changes
    unsigned long long version = 0;
    int adam_t = 0;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kErrParts = 1024;
constexpr int kPoolParts = 32, kPoolChunk = 256;   // partial sums per sample, samples per pass
constexpr long long kIn = mlb::kNetIn;             // input channels of a pool sample

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return mlb::set_error(MLB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

bool plan(mlb_net_s &n, int nx, int ny, int nz, int training)
{
    if (nx < 1 || ny < 1 || nz < 1 || training < 0 || training > 1) return false;
    n.nx = nx; n.ny = ny; n.nz = nz; n.training = training;
    n.N = (long long)nx * ny * nz;
    // the convolution's halo-row offsets are 32-bit site indices, as the
    // lattice's are: the same cap of 2^29 sites
    if (n.N >= (1LL << 29)) return false;
    n.nblk = (int)((n.N + 255) / 256);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
    for (int l = 0; l < mlb::kNetLayers; ++l) {
        auto &L = n.L[l];
        L.cop = mlb::net_cop(l); L.cip = mlb::net_cip(l); L.cout = mlb::net_cout(l); L.cin = mlb::net_cin(l);
        L.nw = 27 * L.cop * L.cip;
        L.w = take(4 * (size_t)L.nw); L.m = take(4 * (size_t)L.nw); L.v = take(4 * (size_t)L.nw);
        // the weight-gradient reduction writes gw and then gb in one row
        L.gw = take(4 * ((size_t)L.nw + L.cop));
        L.gb = L.gw + 4 * (size_t)L.nw;
        L.wb = take(2 * (size_t)L.nw); L.wt = take(2 * (size_t)L.nw);
        L.b = take(4 * (size_t)L.cop); L.mb = take(4 * (size_t)L.cop); L.vb = take(4 * (size_t)L.cop);
    }
    const size_t N = (size_t)n.N;
    n.x = take(2 * (size_t)mlb::kNetInSlots * N);
    for (int l = 0; l < 3; ++l) n.a[l] = take(2 * 32 * N);
    n.y = take(4 * 16 * N);
    n.nc = take(4 * 6 * N);
    n.err = take(8 * 2 * (size_t)kErrParts);
    n.pool = take(8 * (size_t)kPoolParts * kPoolChunk);
    if (training) {
        for (int l = 0; l < 3; ++l) n.z[l] = take(4 * 32 * N);
        n.tg = take(4 * 6 * N);
        n.g3 = take(2 * 16 * N);
        n.g[0] = take(2 * 32 * N);
        n.g[1] = take(2 * 32 * N);
        size_t pf = 0;
        for (int l = 0; l < mlb::kNetLayers; ++l) pf = std::max(pf, mlb::cnn_wgrad_part_floats(l, n.N));
        n.part = take(4 * pf);
        n.loss = take(4 * (size_t)n.nblk);
    }
    n.total = off;
    return true;
}

template <typename T> T *at(const mlb_net_s &n, size_t off) { return reinterpret_cast<T *>(n.ws + off); }

mlb::CnnShape shape_of(const mlb_net_s &n) { return mlb::CnnShape{n.nx, n.ny, n.nz, n.N}; }

// Forward pass from the packed input n.x.  With z buffers (training) the
// pre-activations are kept; the last layer's output goes to n.y.
void forward(mlb_net_s &n, bool keep_z, hipStream_t st)
{
    const mlb::CnnShape sh = shape_of(n);
    const unsigned short *in = at<unsigned short>(n, n.x);
    for (int l = 0; l < mlb::kNetLayers; ++l) {
        const auto &L = n.L[l];
        const bool last = l == mlb::kNetLayers - 1;
        float *z = last ? at<float>(n, n.y) : (keep_z ? at<float>(n, n.z[l]) : nullptr);
        unsigned short *a = last ? nullptr : at<unsigned short>(n, n.a[l]);
        mlb::cnn_conv_fwd(l, sh, in, at<unsigned short>(n, L.wb), at<float>(n, L.b), z, a, last ? 0 : 1, st);
        in = a;
    }
}

mlb_status check_net(mlb_net_s *n)
{
    if (!n) return mlb::set_error(MLB_EINVAL, "null network handle");
    return MLB_OK;
}

}  // namespace

namespace mlb {

int net_grid(const mlb_net_s *n, int *nx, int *ny, int *nz)
{
    *nx = n->nx; *ny = n->ny; *nz = n->nz;
    return 0;
}

unsigned long long net_version(const mlb_net_s *n) { return n->version; }

// the last layer writes the force fields itself (same values as the y
// buffer scaled by f_ref, without the [N][16] round trip)
void net_infer_fields(mlb_net_s *n, const float *dens, const float *mom, float *force, hipStream_t st)
{
    const CnnShape sh = shape_of(*n);
    cnn_pack_input(sh, dens, mom, n->n_ref, n->j_ref, n->f_ref, at<unsigned short>(*n, n->x), st);
    const unsigned short *in = at<unsigned short>(*n, n->x);
    for (int l = 0; l < kNetLayers - 1; ++l) {
        const auto &L = n->L[l];
        unsigned short *a = at<unsigned short>(*n, n->a[l]);
        cnn_conv_fwd(l, sh, in, at<unsigned short>(*n, L.wb), at<float>(*n, L.b), nullptr, a, 1, st);
        in = a;
    }
    const auto &L = n->L[kNetLayers - 1];
    cnn_conv_out_fields(sh, in, at<unsigned short>(*n, L.wb), at<float>(*n, L.b), n->f_ref, force, st);
}

float *net_check_buffer(mlb_net_s *n) { return at<float>(*n, n->nc); }
double *net_err_buffer(mlb_net_s *n, int *nparts)
{
    *nparts = kErrParts;
    return at<double>(*n, n->err);
}

void net_sample(mlb_net_s *n, const float *dens, const float *mom, const float *force, float *x_out,
                float *target_out, hipStream_t st)
{
    cnn_fields_x(shape_of(*n), dens, mom, n->n_ref, n->j_ref, force, n->f_ref, x_out, target_out, st);
}

}  // namespace mlb

extern "C" {

size_t mlb_net_param_count(void)
{
    size_t c = 0;
    for (int l = 0; l < mlb::kNetLayers; ++l)
        c += (size_t)27 * mlb::net_cout(l) * mlb::net_cin(l) + mlb::net_cout(l);
    return c;
}

size_t mlb_net_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t training)
{
    mlb_net_s n;
    if (!plan(n, nx, ny, nz, training)) return 0;
    return n.total;
}

mlb_status mlb_net_create(int32_t nx, int32_t ny, int32_t nz, int32_t training, void *workspace,
                          size_t workspace_bytes, void *stream, mlb_net *out)
{
    if (!out) return mlb::set_error(MLB_EINVAL, "out is null");
    *out = nullptr;
    mlb_net_s tmp;
    if (!plan(tmp, nx, ny, nz, training)) return mlb::set_error(MLB_EINVAL, "invalid network grid or flag");
    if (!workspace || workspace_bytes < tmp.total)
        return mlb::set_error(MLB_EINVAL, "network workspace missing or too small (need " +
                                              std::to_string(tmp.total) + " bytes)");
    if (!mlb::cnn_prepare()) return mlb::set_error(MLB_EHIP, "cannot raise the LDS limit of the convolution kernels");
    auto *n = new mlb_net_s(tmp);
    n->ws = static_cast<char *>(workspace);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // zero parameters and moments (padded entries stay zero for good)
    for (int l = 0; l < mlb::kNetLayers; ++l) {
        const auto &L = n->L[l];
        const size_t bytes = L.vb + 4 * (size_t)L.cop - L.w;
        hipError_t e = hipMemsetAsync(n->ws + L.w, 0, bytes, st);
        if (e != hipSuccess) {
            delete n;
            return mlb::set_error(MLB_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
        }
    }
    *out = n;
    return MLB_OK;
}

mlb_status mlb_net_set_params(mlb_net n, const float *params, void *stream)
{
    if (mlb_status s = check_net(n)) return s;
    if (!params) return mlb::set_error(MLB_EINVAL, "params is null");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float *p = params;
    for (int l = 0; l < mlb::kNetLayers; ++l) {
        const auto &L = n->L[l];
        std::vector<float> w((size_t)L.nw, 0.f), b((size_t)L.cop, 0.f);
        for (int co = 0; co < L.cout; ++co)
            for (int ci = 0; ci < L.cin; ++ci)
                for (int t = 0; t < 27; ++t) w[((size_t)t * L.cop + co) * L.cip + ci] = *p++;
        for (int co = 0; co < L.cout; ++co) b[co] = *p++;
        HIP_TRY(hipMemcpyAsync(n->ws + L.w, w.data(), 4 * w.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(n->ws + L.b, b.data(), 4 * b.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemsetAsync(n->ws + L.m, 0, 4 * (size_t)L.nw, st));
        HIP_TRY(hipMemsetAsync(n->ws + L.v, 0, 4 * (size_t)L.nw, st));
        HIP_TRY(hipMemsetAsync(n->ws + L.mb, 0, 4 * (size_t)L.cop, st));
        HIP_TRY(hipMemsetAsync(n->ws + L.vb, 0, 4 * (size_t)L.cop, st));
        mlb::cnn_cast(L.nw, L.cop, L.cip, at<float>(*n, L.w), at<unsigned short>(*n, L.wb),
                      at<unsigned short>(*n, L.wt), st);
    }
    n->adam_t = 0;
    HIP_TRY(hipGetLastError());
    // the host vectors above must outlive the copies
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

mlb_status mlb_net_get_params(mlb_net n, float *params, void *stream)
{
    if (mlb_status s = check_net(n)) return s;
    if (!params) return mlb::set_error(MLB_EINVAL, "params is null");
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *p = params;
    for (int l = 0; l < mlb::kNetLayers; ++l) {
        const auto &L = n->L[l];
        std::vector<float> w((size_t)L.nw), b((size_t)L.cop);
        HIP_TRY(hipMemcpyAsync(w.data(), n->ws + L.w, 4 * w.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(b.data(), n->ws + L.b, 4 * b.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int co = 0; co < L.cout; ++co)
            for (int ci = 0; ci < L.cin; ++ci)
                for (int t = 0; t < 27; ++t) *p++ = w[((size_t)t * L.cop + co) * L.cip + ci];
        for (int co = 0; co < L.cout; ++co) *p++ = b[co];
    }
    return MLB_OK;
}

mlb_status mlb_net_set_scales(mlb_net n, double n_ref, double j_ref, double f_ref)
{
    if (mlb_status s = check_net(n)) return s;
    if (!(n_ref > 0) || !(j_ref > 0) || !(f_ref > 0) || !std::isfinite(n_ref) || !std::isfinite(j_ref) ||
        !std::isfinite(f_ref))
        return mlb::set_error(MLB_EINVAL, "scales must be positive and finite");
    n->n_ref = (float)n_ref;
    n->j_ref = (float)j_ref;
    n->f_ref = (float)f_ref;
    n->version += 1;
    return MLB_OK;
}

namespace {
// float64 sums of squares over `len` floats at base + s stride for samples
// s = 0..count-1 (partials on the GPU, added on the host in fixed order)
mlb_status pool_sumsq(mlb_net_s &n, const float *base, long long stride, long long len, int count, double *out,
                      hipStream_t st)
{
    std::vector<double> h((size_t)kPoolParts * kPoolChunk);
    double *part = at<double>(n, n.pool);
    for (int s0 = 0; s0 < count; s0 += kPoolChunk) {
        const int c = std::min(kPoolChunk, count - s0);
        mlb::cnn_pool_sumsq(base + (long long)s0 * stride, stride, len, c, part, kPoolParts, st);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * kPoolParts * c, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int s = 0; s < c; ++s) {
            double acc = 0.0;
            for (int p = 0; p < kPoolParts; ++p) acc += h[(size_t)s * kPoolParts + p];
            out[s0 + s] = acc;
        }
    }
    return MLB_OK;
}
}  // namespace

mlb_status mlb_net_pool_stats(mlb_net n, const float *x, const float *t, int32_t count, double *out, void *stream)
{
    if (mlb_status s = check_net(n)) return s;
    if (!x || !t || !out || count < 1) return mlb::set_error(MLB_EINVAL, "x, t, out and count >= 1 are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long N = n->N;
    std::vector<double> sx((size_t)count), stt((size_t)count);
    // the momentum channels 2..7 of every input sample
    if (mlb_status s = pool_sumsq(*n, x + 2 * N, kIn * N, 6 * N, count, sx.data(), st)) return s;
    if (mlb_status s = pool_sumsq(*n, t, 6 * N, 6 * N, count, stt.data(), st)) return s;
    double jx = 0.0;
    for (int s = 0; s < count; ++s) jx += sx[(size_t)s];
    out[0] = jx / (6.0 * (double)N * count);
    for (int s = 0; s < count; ++s) out[1 + s] = stt[(size_t)s] / (6.0 * (double)N);
    return MLB_OK;
}

mlb_status mlb_net_pool_rescale(mlb_net n, float *x, float *t, int32_t count, double j_div, double f_div, void *stream)
{
    if (mlb_status s = check_net(n)) return s;
    if (!x || !t || count < 1) return mlb::set_error(MLB_EINVAL, "x, t and count >= 1 are required");
    if (!(j_div > 0) || !(f_div > 0) || !std::isfinite(j_div) || !std::isfinite(f_div))
        return mlb::set_error(MLB_EINVAL, "divisors must be positive and finite");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long N = n->N;
    for (int s0 = 0; s0 < count; s0 += kPoolChunk) {       // grid.y stays within its limit
        const int c = std::min(kPoolChunk, count - s0);
        mlb::cnn_pool_scale(x + 2 * N + (long long)s0 * kIn * N, kIn * N, 6 * N, c, (float)(1.0 / j_div), st);
        mlb::cnn_pool_scale(x + 8 * N + (long long)s0 * kIn * N, kIn * N, 6 * N, c, (float)(1.0 / f_div), st);
        mlb::cnn_pool_scale(t + (long long)s0 * 6 * N, 6 * N, 6 * N, c, (float)(1.0 / f_div), st);
        HIP_TRY(hipGetLastError());
    }
    return MLB_OK;
}

mlb_status mlb_net_rel_error(mlb_net n, const float *y, const float *t, double *err, void *stream)
{
    if (mlb_status s = check_net(n)) return s;
    if (!y || !t || !err) return mlb::set_error(MLB_EINVAL, "y, t and err are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = at<double>(*n, n->err);
    mlb::cnn_err_partial(6 * n->N, y, t, part, kErrParts, st);
    HIP_TRY(hipGetLastError());
    std::vector<double> h(2 * (size_t)kErrParts);
    HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double e = 0.0, w = 0.0;
    for (int p = 0; p < kErrParts; ++p) {
        e += h[2 * (size_t)p];
        w += h[2 * (size_t)p + 1];
    }
    *err = w > 0.0 ? std::sqrt(e / w) : (e > 0.0 ? INFINITY : 0.0);
    return MLB_OK;
}

mlb_status mlb_net_forward(mlb_net n, const float *x, float *y, void *stream)
{
    if (mlb_status s = check_net(n)) return s;
    if (!x || !y) return mlb::set_error(MLB_EINVAL, "x and y must be device pointers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const mlb::CnnShape sh = shape_of(*n);
    mlb::cnn_pack_x(sh, x, at<unsigned short>(*n, n->x), st);
    forward(*n, false, st);
    mlb::cnn_unpack_output(sh, at<float>(*n, n->y), 1.f, y, st);
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status mlb_net_train_step(mlb_net n, const float *x, const float *target, float lr, float loss_weight, int32_t update,
                              double *loss, float *grads, void *stream)
{
    if (mlb_status s = check_net(n)) return s;
    if (!n->training) return mlb::set_error(MLB_ESTATE, "network was created without training buffers");
    if (!x || !target) return mlb::set_error(MLB_EINVAL, "x and target must be device pointers");
    if (update && !(lr >= 0.f && std::isfinite(lr))) return mlb::set_error(MLB_EINVAL, "lr must be >= 0");
    if (!(loss_weight > 0.f && std::isfinite(loss_weight)))
        return mlb::set_error(MLB_EINVAL, "loss_weight must be positive and finite");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const mlb::CnnShape sh = shape_of(*n);
    mlb::cnn_pack_x(sh, x, at<unsigned short>(*n, n->x), st);
    mlb::cnn_pack_target(sh, target, 1.f, at<float>(*n, n->tg), st);
    forward(*n, true, st);
    mlb::cnn_mse(sh, loss_weight, at<float>(*n, n->y), at<float>(*n, n->tg), at<unsigned short>(*n, n->g3),
                 at<float>(*n, n->loss), st);
    // backward: gradient w.r.t. the pre-activation of layer l in gz
    const unsigned short *gz = at<unsigned short>(*n, n->g3);
    for (int l = mlb::kNetLayers - 1; l >= 0; --l) {
        const auto &L = n->L[l];
        const unsigned short *ain = l == 0 ? at<unsigned short>(*n, n->x) : at<unsigned short>(*n, n->a[l - 1]);
        mlb::cnn_conv_wgrad(l, sh, gz, ain, at<float>(*n, n->part), at<float>(*n, L.gw), st);
        if (l > 0) {
            unsigned short *gin = at<unsigned short>(*n, n->g[l & 1]);
            mlb::cnn_conv_dgrad(l, sh, gz, at<unsigned short>(*n, L.wt), at<float>(*n, n->z[l - 1]), gin, st);
            gz = gin;
        }
    }
    if (update) {
        n->adam_t += 1;
        for (int l = 0; l < mlb::kNetLayers; ++l) {
            const auto &L = n->L[l];
            mlb::cnn_adam(L.nw, L.cop, L.cip, L.cout, L.cin, at<float>(*n, L.w), at<float>(*n, L.gw),
                          at<float>(*n, L.m), at<float>(*n, L.v), lr, 0.9, 0.999, 1e-8, n->adam_t,
                          at<unsigned short>(*n, L.wb), at<unsigned short>(*n, L.wt), at<float>(*n, L.b),
                          at<float>(*n, L.gb), at<float>(*n, L.mb), at<float>(*n, L.vb), st);
        }
    }
    HIP_TRY(hipGetLastError());
    if (loss) {
        std::vector<float> lp((size_t)n->nblk);
        HIP_TRY(hipMemcpyAsync(lp.data(), n->ws + n->loss, 4 * lp.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double s = 0.0;
        for (float v : lp) s += (double)v;
        *loss = s / ((double)n->N * mlb::kNetOut);
    }
    if (grads) {
        float *p = grads;
        for (int l = 0; l < mlb::kNetLayers; ++l) {
            const auto &L = n->L[l];
            std::vector<float> w((size_t)L.nw), b((size_t)L.cop);
            HIP_TRY(hipMemcpyAsync(w.data(), n->ws + L.gw, 4 * w.size(), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(b.data(), n->ws + L.gb, 4 * b.size(), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            for (int co = 0; co < L.cout; ++co)
                for (int ci = 0; ci < L.cin; ++ci)
                    for (int t = 0; t < 27; ++t) *p++ = w[((size_t)t * L.cop + co) * L.cip + ci];
            for (int co = 0; co < L.cout; ++co) *p++ = b[co];
        }
    }
    return MLB_OK;
}

int32_t mlb_net_adam_steps(mlb_net n) { return n ? n->adam_t : -1; }

mlb_status mlb_net_destroy(mlb_net n)
{
    delete n;
    return MLB_OK;
}

}  // extern "C"
