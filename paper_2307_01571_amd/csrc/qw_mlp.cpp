// qw_mlp.cpp -- host engine of the surrogate network (qw_mlp_* in qw_mlp.h):
// workspace carving and the launch sequences of the forward pass, the
// back-propagation and the Adam step.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qw.h"
#include "qw_mlp.h"
#include "qw_host.hpp"
#include "qw_mlp_launch.hpp"

// Scratch of qw_mlp_predict_static: the inputs and activations of one
// prediction, in a device array of the library rather than the caller's
// workspace (each GPU the library runs on holds its own copy until the
// process ends).  Host code must not pass `scratch` itself to a kernel (on
// the host it names a stand-in, not device memory): it uses the address
// hipGetSymbolAddress gives for the device, kept per device below.
constexpr size_t kScratchBytes = (size_t)QW_MLP_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

using qwm::kInPad;

constexpr size_t kAlign = 256;
constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int round64(int v) { return (v + 63) / 64 * 64; }

struct Layer {
    int n_out, n_in, in_pad, out_pad;
    long long p_off, b_off;  // weights and bias in the flat parameters of one net
    long long wb_off, wt_off;
};

struct Plan {
    qw_mlp_shape s{};
    int L = 0;             // linear layers = depth + 1
    long long np = 0;      // parameters per net
    long long nwb = 0;     // bfloat16 weight elements per net (each layout)
    int Mpad = 0;          // batch rows, padded
    std::vector<Layer> layer;
    // byte offsets
    size_t P, Mo, V, G, Wb, Wt, shift, scale, oshift, oscale, swt, Xb, Xt, Z, H, Ht, Y, dYb, dYt, dZb, dZt, loss_part, loss;
    size_t Kp;             // split-K parts of the weight gradients
    int ks_max = 1;        // most K splits of a weight-gradient product
    long long kp_net = 0;  // floats per net in Kp
    size_t total;
};

int check_shape(const qw_mlp_shape* s, std::string* msg)
{
    if (!s) {
        *msg = "shape is NULL";
        return QW_E_ARG;
    }
    if (s->n_in < 1 || s->n_in > kInPad || s->n_out < 1 || s->n_out > kInPad || s->depth < 1 || s->depth > 16 ||
        s->n_nets < 1 || s->n_nets > 16 || s->max_batch < 1 || s->max_batch > 65536 || s->width < 64 ||
        s->width > 1024 || s->width % 64 != 0) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "shape n_in=%d width=%d depth=%d n_out=%d n_nets=%d max_batch=%d outside the supported range",
                 s->n_in, s->width, s->depth, s->n_out, s->n_nets, s->max_batch);
        *msg = buf;
        return QW_E_SIZE;
    }
    return QW_OK;
}

Plan make_plan(const qw_mlp_shape& s)
{
    Plan p;
    p.s = s;
    p.L = s.depth + 1;
    p.Mpad = round64(s.max_batch);
    long long o = 0, w = 0;
    for (int l = 0; l < p.L; ++l) {
        Layer y;
        y.n_in = l == 0 ? s.n_in : s.width;
        y.n_out = l == p.L - 1 ? s.n_out : s.width;
        y.in_pad = l == 0 ? kInPad : s.width;
        y.out_pad = l == p.L - 1 ? kInPad : s.width;
        y.p_off = o;
        o += (long long)y.n_out * y.n_in;
        y.b_off = o;
        o += y.n_out;
        y.wb_off = w;
        y.wt_off = w;
        w += (long long)y.out_pad * y.in_pad;
        p.layer.push_back(y);
    }
    p.np = o;
    p.nwb = w;
    const long long nets = s.n_nets, M = p.Mpad, W = s.width, D = s.depth;
    size_t b = 0;
    auto take = [&](size_t bytes) {
        const size_t at = b;
        b = align_up(b + bytes);
        return at;
    };
    p.P = take(4 * nets * p.np);
    p.Mo = take(4 * nets * p.np);
    p.V = take(4 * nets * p.np);
    p.G = take(4 * nets * p.np);
    p.Wb = take(2 * nets * p.nwb);
    p.Wt = take(2 * nets * p.nwb);
    p.shift = take(4 * kInPad);
    p.scale = take(4 * kInPad);
    p.oshift = take(4 * kInPad);
    p.oscale = take(4 * kInPad);
    p.swt = take(4 * kInPad);
    p.Xb = take(2 * M * kInPad);
    p.Xt = take(2 * M * kInPad);
    p.Z = take(4 * nets * D * M * W);
    p.H = take(2 * nets * D * M * W);
    p.Ht = take(2 * nets * D * M * W);
    p.Y = take(4 * nets * M * kInPad);
    p.dYb = take(2 * nets * M * kInPad);
    p.dYt = take(2 * nets * M * kInPad);
    p.dZb = take(2 * nets * 2 * M * W);
    p.dZt = take(2 * nets * 2 * M * W);
    p.loss_part = take(4 * nets * (M / 64));
    p.loss = take(4 * nets);
    // weight gradients sum over the batch (K = batch rows) on few output
    // tiles: split K so that each net's product covers about 256 workgroups
    // (independent of the number of nets, so a net's gradients do not
    // depend on the ensemble it is trained in)
    long long wmax = 0;
    for (const Layer& y : p.layer) wmax = std::max(wmax, (long long)y.n_out * y.n_in);
    const long long tiles = (W / 64) * (W / 64);
    p.ks_max = (int)std::max(1LL, std::min(16LL, 256 / tiles));
    p.kp_net = p.ks_max > 1 ? p.ks_max * wmax : 0;
    p.Kp = take(4 * nets * p.kp_net);
    p.total = b;
    return p;
}

}  // namespace

struct qw_mlp_s {
    Plan p;
    char* ws = nullptr;
    int device = 0;   // the workspace's device
    long long t = 0;  // Adam steps taken
    std::string err;
};

namespace {

thread_local std::string g_mlp_error;

int mfail(qw_mlp h, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_mlp_error = buf;
    return code;
}

int mhip(qw_mlp h, hipError_t e, const char* what) { return mfail(h, QW_E_DEVICE, "%s: %s", what, hipGetErrorString(e)); }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
T* at(qw_mlp h, size_t off)
{
    return reinterpret_cast<T*>(h->ws + off);
}

qwm::AdamArgs adam_args(qw_mlp h, int update, float lr)
{
    const Plan& p = h->p;
    qwm::AdamArgs a{};
    a.p = at<float>(h, p.P);
    a.m = at<float>(h, p.Mo);
    a.v = at<float>(h, p.V);
    a.g = at<float>(h, p.G);
    a.n = (int)p.np;
    a.update = update;
    a.lr = lr;
    a.b1 = kB1;
    a.b2 = kB2;
    a.eps = kEps;
    if (update) {
        a.c1 = (float)(1.0 / (1.0 - std::pow((double)kB1, (double)h->t)));
        a.c2 = (float)(1.0 / (1.0 - std::pow((double)kB2, (double)h->t)));
    }
    a.wb = at<__bf16>(h, p.Wb);
    a.wt = at<__bf16>(h, p.Wt);
    a.s_wb = p.nwb;
    a.s_wt = p.nwb;
    a.n_layers = p.L;
    for (int l = 0; l < p.L; ++l) {
        const Layer& y = p.layer[l];
        a.layer[l] = qwm::LayerMap{(int)y.p_off, y.n_out, y.n_in, (int)y.wb_off, y.in_pad, (int)y.wt_off, y.out_pad};
    }
    return a;
}

// Forward pass of every net for B samples.  With t (targets) the training
// outputs are kept: pre-activations, transposed activations, dY and the loss
// partials.
// Where a forward pass keeps its inputs and activations: the workspace's
// buffers (rows M = the padded maximum batch), or the static scratch array
// of qw_mlp_predict_static (rows M = its padded batch).
struct Act {
    __bf16 *Xb, *Xt, *H;
    float* Y;
    int M;
};

Act ws_act(qw_mlp h)
{
    const Plan& p = h->p;
    return {at<__bf16>(h, p.Xb), at<__bf16>(h, p.Xt), at<__bf16>(h, p.H), at<float>(h, p.Y), p.Mpad};
}

// bytes of the activation buffers for M rows, each region 256-aligned, and their offsets
struct ActLayout {
    size_t xb, xt, hh, y, total;
};
ActLayout act_layout(const Plan& p, int M)
{
    const size_t nets = p.s.n_nets, W = p.s.width, D = p.s.depth;
    ActLayout a{};
    size_t o = 0;
    a.xb = o;
    o = align_up(o + 2 * (size_t)M * kInPad);
    a.xt = o;
    o = align_up(o + 2 * (size_t)M * kInPad);
    a.hh = o;
    o = align_up(o + 2 * nets * D * M * W);
    a.y = o;
    o = align_up(o + 4 * nets * M * kInPad);
    a.total = o;
    return a;
}

// training (t != NULL) needs the workspace's activations (a.M == Mpad)
hipError_t forward(qw_mlp h, const Act& a, const float* x, const float* t, int B, hipStream_t s)
{
    const Plan& p = h->p;
    const int W = p.s.width, D = p.s.depth, M = a.M, nets = p.s.n_nets;
    const int Mp = round64(B);
    const bool train = t != nullptr;
    hipError_t e = qwm::launch_prep_input(x, B, p.s.n_in, Mp, at<float>(h, p.shift), at<float>(h, p.scale), a.Xb,
                                          a.Xt, s);
    // note: Xt rows are Mp long here (ld = Mp); the products below read them with ld = Mp
    const long long sAct = (long long)D * M * W;  // per-net stride of Z, H, Ht
    for (int l = 0; l < D && e == hipSuccess; ++l) {
        const Layer& y = p.layer[l];
        qwm::GemmArgs g{};
        if (l == 0) {
            g.A = a.Xb;
            g.sA = 0;
            g.lda = kInPad;
        } else {
            g.A = a.H + (size_t)(l - 1) * M * W;
            g.sA = sAct;
            g.lda = W;
        }
        g.B = at<__bf16>(h, p.Wb) + y.wb_off;
        g.sB = p.nwb;
        g.ldb = y.in_pad;
        g.M = B;
        g.N = W;
        g.K = y.in_pad;
        g.Mpad = Mp;
        g.bias = at<float>(h, p.P) + y.b_off;
        g.sbias = p.np;
        if (train) {
            g.Cf = at<float>(h, p.Z) + (size_t)l * M * W;
            g.sCf = sAct;
            g.ldcf = W;
            g.Ct = at<__bf16>(h, p.Ht) + (size_t)l * M * W;
            g.sCt = sAct;
            g.ldct = Mp;
            g.nct = W;
        }
        g.Cb = a.H + (size_t)l * M * W;
        g.sCb = sAct;
        g.ldcb = W;
        e = qwm::launch_gemm(qwm::EPI_HIDDEN, g, nets, W, s);
    }
    if (e != hipSuccess) return e;
    const Layer& y = p.layer[D];
    qwm::GemmArgs g{};
    g.A = a.H + (size_t)(D - 1) * M * W;
    g.sA = sAct;
    g.lda = W;
    g.B = at<__bf16>(h, p.Wb) + y.wb_off;
    g.sB = p.nwb;
    g.ldb = W;
    g.M = B;
    g.N = p.s.n_out;
    g.K = W;
    g.Mpad = Mp;
    g.bias = at<float>(h, p.P) + y.b_off;
    g.sbias = p.np;
    g.Cf = a.Y;
    g.sCf = (long long)M * kInPad;
    g.ldcf = kInPad;
    if (train) {
        g.T = t;
        g.ldt = p.s.n_out;
        g.gscale = 2.0f / ((float)B * (float)p.s.n_out);
        g.Cb = at<__bf16>(h, p.dYb);
        g.sCb = (long long)M * kInPad;
        g.ldcb = kInPad;
        g.Ct = at<__bf16>(h, p.dYt);
        g.sCt = (long long)M * kInPad;
        g.ldct = Mp;
        g.nct = kInPad;
        g.loss_part = at<float>(h, p.loss_part);
        g.sLoss = M / 64;
    }
    e = qwm::launch_gemm(qwm::EPI_OUT, g, nets, kInPad, s);
    if (e == hipSuccess && train)
        e = qwm::launch_loss_finish(at<float>(h, p.loss_part), M / 64, Mp / 64, 1.0f / ((float)B * p.s.n_out),
                                    at<float>(h, p.loss), nets, s);
    return e;
}

// weight gradient dW[out][in] = sum_m dZt[out][m] Ht[in][m] (+ bias gradient as row sums of dZt)
hipError_t weight_grad(qw_mlp h, int l, const __bf16* dzt, long long s_dzt, const __bf16* ht, long long s_ht,
                       int Mp, int B, hipStream_t s)
{
    const Plan& p = h->p;
    const Layer& y = p.layer[l];
    qwm::GemmArgs g{};
    g.A = dzt;
    g.sA = s_dzt;
    g.lda = Mp;
    g.B = ht;
    g.sB = s_ht;
    g.ldb = Mp;
    g.M = y.n_out;
    g.N = y.n_in;
    g.K = Mp;
    g.Mpad = round64(y.n_out);
    float* dw = at<float>(h, p.G) + y.p_off;
    // split K (the batch) into chunks of at least 256 rows, multiples of 64
    int ks = std::min(p.ks_max, Mp / 256);
    hipError_t e;
    if (ks >= 2) {
        const int chunk = round64((Mp + ks - 1) / ks);
        ks = (Mp + chunk - 1) / chunk;
        g.ksplit = ks;
        g.k_chunk = chunk;
        g.Cp = at<float>(h, p.Kp);
        g.sCp_net = p.kp_net;
        e = qwm::launch_gemm(qwm::EPI_PARTIAL, g, p.s.n_nets, y.n_in, s);
        // the parts' sum and the bias gradient (row sums of dZ^T) in one launch
        if (e == hipSuccess)
            e = qwm::launch_ksum_rows(g.Cp, p.kp_net, ks, y.n_out, y.n_in, dw, p.np, y.n_in, dzt, s_dzt, Mp, y.n_out,
                                      B, at<float>(h, p.G) + y.b_off, p.np, p.s.n_nets, s);
        return e;
    }
    g.Cf = dw;
    g.sCf = p.np;
    g.ldcf = y.n_in;
    e = qwm::launch_gemm(qwm::EPI_F32, g, p.s.n_nets, y.n_in, s);
    if (e == hipSuccess)
        e = qwm::launch_row_sums(dzt, s_dzt, Mp, y.n_out, B, at<float>(h, p.G) + y.b_off, p.np, p.s.n_nets, s);
    return e;
}

// dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1}) from dZ_l [B][kpad] (row-major) and Wt_l
hipError_t act_grad(qw_mlp h, int l, const __bf16* dzb, long long s_dzb, int lda, __bf16* out_b, __bf16* out_t,
                    long long s_out, int Mp, int B, hipStream_t s)
{
    const Plan& p = h->p;
    const Layer& y = p.layer[l];
    const int W = p.s.width, M = p.Mpad;
    qwm::GemmArgs g{};
    g.A = dzb;
    g.sA = s_dzb;
    g.lda = lda;
    g.B = at<__bf16>(h, p.Wt) + y.wt_off;
    g.sB = p.nwb;
    g.ldb = y.out_pad;
    g.M = B;
    g.N = W;
    g.K = y.out_pad;
    g.Mpad = Mp;
    g.Z = at<float>(h, p.Z) + (size_t)(l - 1) * M * W;
    g.sZ = (long long)p.s.depth * M * W;
    g.ldz = W;
    g.Cb = out_b;
    g.sCb = s_out;
    g.ldcb = W;
    g.Ct = out_t;
    g.sCt = s_out;
    g.ldct = Mp;
    g.nct = W;
    return qwm::launch_gemm(qwm::EPI_GELU_BWD, g, p.s.n_nets, W, s);
}

hipError_t backward(qw_mlp h, int B, hipStream_t s)
{
    const Plan& p = h->p;
    const int W = p.s.width, D = p.s.depth, M = p.Mpad;
    const int Mp = round64(B);
    const long long sAct = (long long)D * M * W;
    const long long sY = (long long)M * kInPad;
    const long long sdz = 2LL * M * W;
    // output layer
    hipError_t e = weight_grad(h, D, at<__bf16>(h, p.dYt), sY, at<__bf16>(h, p.Ht) + (size_t)(D - 1) * M * W, sAct,
                               Mp, B, s);
    int cur = 0;
    if (e == hipSuccess)
        e = act_grad(h, D, at<__bf16>(h, p.dYb), sY, kInPad, at<__bf16>(h, p.dZb), at<__bf16>(h, p.dZt), sdz, Mp, B, s);
    for (int l = D - 1; l >= 1 && e == hipSuccess; --l) {
        const __bf16* dzt = at<__bf16>(h, p.dZt) + (size_t)cur * M * W;
        const __bf16* dzb = at<__bf16>(h, p.dZb) + (size_t)cur * M * W;
        e = weight_grad(h, l, dzt, sdz, at<__bf16>(h, p.Ht) + (size_t)(l - 1) * M * W, sAct, Mp, B, s);
        const int nxt = 1 - cur;
        if (e == hipSuccess)
            e = act_grad(h, l, dzb, sdz, W, at<__bf16>(h, p.dZb) + (size_t)nxt * M * W,
                         at<__bf16>(h, p.dZt) + (size_t)nxt * M * W, sdz, Mp, B, s);
        cur = nxt;
    }
    if (e == hipSuccess)
        e = weight_grad(h, 0, at<__bf16>(h, p.dZt) + (size_t)cur * M * W, sdz, at<__bf16>(h, p.Xt), 0, Mp, B, s);
    return e;
}

// per-device addresses of `scratch`, looked up once per device with that
// device current (qw_mlp_init), read by qw_mlp_predict_static
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != device) e = hipSetDevice(device);
    void* ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e == hipSuccess && !ptr) e = hipErrorInvalidSymbol;
    if (e == hipSuccess) g_scratch_ptr[device] = ptr;
    return e;
}

void* scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

int check_batch(qw_mlp h, const float* x, int B)
{
    if (!h) return mfail(nullptr, QW_E_ARG, "network is NULL");
    if (!x) return mfail(h, QW_E_ARG, "x is NULL");
    if (B < 1 || B > h->p.s.max_batch) return mfail(h, QW_E_ARG, "batch %d outside [1, %d]", B, h->p.s.max_batch);
    return QW_OK;
}

}  // namespace

extern "C" {

int qw_mlp_param_count(const qw_mlp_shape* s, int64_t* per_net)
{
    std::string msg;
    const int rc = check_shape(s, &msg);
    if (rc != QW_OK) return mfail(nullptr, rc, "%s", msg.c_str());
    if (!per_net) return mfail(nullptr, QW_E_ARG, "per_net is NULL");
    *per_net = make_plan(*s).np;
    return QW_OK;
}

int qw_mlp_workspace_bytes(const qw_mlp_shape* s, size_t* bytes)
{
    std::string msg;
    const int rc = check_shape(s, &msg);
    if (rc != QW_OK) return mfail(nullptr, rc, "%s", msg.c_str());
    if (!bytes) return mfail(nullptr, QW_E_ARG, "bytes is NULL");
    *bytes = make_plan(*s).total;
    return QW_OK;
}

int qw_mlp_init(qw_mlp* out, const qw_mlp_shape* s, const float* shift, const float* scale, void* workspace,
                size_t ws_bytes, void* hip_stream)
{
    if (!out) return mfail(nullptr, QW_E_ARG, "out is NULL");
    *out = nullptr;
    std::string msg;
    int rc = check_shape(s, &msg);
    if (rc != QW_OK) return mfail(nullptr, rc, "%s", msg.c_str());
    if (!shift || !scale) return mfail(nullptr, QW_E_ARG, "shift or scale is NULL");
    for (int i = 0; i < s->n_in; ++i)
        if (!std::isfinite(shift[i]) || !std::isfinite(scale[i]))
            return mfail(nullptr, QW_E_ARG, "input map entry %d is not finite", i);
    if (!workspace) return mfail(nullptr, QW_E_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return mfail(nullptr, QW_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    Plan p = make_plan(*s);
    if (ws_bytes < p.total)
        return mfail(nullptr, QW_E_WORKSPACE, "workspace has %zu bytes, the network needs %zu", ws_bytes, p.total);
    int ws_device = 0;
    {
        std::string msg;
        const int drc = qwh::device_of(workspace, &ws_device, &msg);
        if (drc != QW_OK) return mfail(nullptr, drc, "%s", msg.c_str());
    }
    {
        const hipError_t se = scratch_setup(ws_device);
        if (se != hipSuccess)
            return mfail(nullptr, QW_E_DEVICE, "static scratch of device %d: %s", ws_device, hipGetErrorString(se));
    }
    qw_mlp h = new (std::nothrow) qw_mlp_s;
    if (!h) return mfail(nullptr, QW_E_DEVICE, "out of host memory");
    h->p = p;
    h->ws = static_cast<char*>(workspace);
    h->device = ws_device;
    hipStream_t st = as_stream(hip_stream);
    float map[5 * kInPad] = {};
    for (int i = 0; i < s->n_in; ++i) {
        map[i] = shift[i];
        map[kInPad + i] = scale[i];
    }
    for (int i = 0; i < kInPad; ++i) map[3 * kInPad + i] = 1.0f;  // output map: identity
    for (int i = 0; i < kInPad; ++i) map[4 * kInPad + i] = 1.0f;  // spread weights: one
    // zero everything (the paddings of weights and activations must read as zero)
    hipError_t e = qwm::launch_fill_zero(h->ws, p.total, st);
    if (e == hipSuccess) e = hipMemcpyAsync(at<float>(h, p.shift), map, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<float>(h, p.scale), map + kInPad, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<float>(h, p.oshift), map + 2 * kInPad, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<float>(h, p.oscale), map + 3 * kInPad, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<float>(h, p.swt), map + 4 * kInPad, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        mfail(nullptr, QW_E_DEVICE, "network set-up: %s", hipGetErrorString(e));
        delete h;
        return QW_E_DEVICE;
    }
    *out = h;
    return QW_OK;
}

int qw_mlp_set_params(qw_mlp h, const float* params, void* hip_stream)
{
    if (!h) return mfail(nullptr, QW_E_ARG, "network is NULL");
    if (!params) return mfail(h, QW_E_ARG, "params is NULL");
    const Plan& p = h->p;
    hipStream_t s = as_stream(hip_stream);
    const size_t bytes = 4 * (size_t)p.s.n_nets * p.np;
    hipError_t e = hipMemcpyAsync(at<float>(h, p.P), params, bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = qwm::launch_fill_zero(at<float>(h, p.Mo), bytes, s);
    if (e == hipSuccess) e = qwm::launch_fill_zero(at<float>(h, p.V), bytes, s);
    if (e == hipSuccess) e = qwm::launch_adam(adam_args(h, 0, 0.0f), p.s.n_nets, s);
    if (e != hipSuccess) return mhip(h, e, "set params");
    h->t = 0;
    return QW_OK;
}

int qw_mlp_set_output_map(qw_mlp h, const float* shift, const float* scale, void* hip_stream)
{
    if (!h) return mfail(nullptr, QW_E_ARG, "network is NULL");
    if (!shift || !scale) return mfail(h, QW_E_ARG, "shift or scale is NULL");
    float map[2 * kInPad] = {};
    for (int i = 0; i < kInPad; ++i) map[kInPad + i] = 1.0f;
    for (int i = 0; i < h->p.s.n_out; ++i) {
        if (!std::isfinite(shift[i]) || !std::isfinite(scale[i]))
            return mfail(h, QW_E_ARG, "output map entry %d is not finite", i);
        map[i] = shift[i];
        map[kInPad + i] = scale[i];
    }
    hipStream_t st = as_stream(hip_stream);
    hipError_t e = hipMemcpyAsync(at<float>(h, h->p.oshift), map, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<float>(h, h->p.oscale), map + kInPad, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return mhip(h, e, "output map");
    return QW_OK;
}

int qw_mlp_set_spread_weights(qw_mlp h, const float* w, void* hip_stream)
{
    if (!h) return mfail(nullptr, QW_E_ARG, "network is NULL");
    if (!w) return mfail(h, QW_E_ARG, "weights are NULL");
    float buf[kInPad] = {};
    for (int i = 0; i < h->p.s.n_out; ++i) {
        if (!std::isfinite(w[i]) || w[i] < 0.0f) return mfail(h, QW_E_ARG, "spread weight %d is not finite and >= 0", i);
        buf[i] = w[i];
    }
    hipStream_t st = as_stream(hip_stream);
    hipError_t e = hipMemcpyAsync(at<float>(h, h->p.swt), buf, 4 * kInPad, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return mhip(h, e, "spread weights");
    return QW_OK;
}

int qw_mlp_get_params(qw_mlp h, float* params, void* hip_stream)
{
    if (!h) return mfail(nullptr, QW_E_ARG, "network is NULL");
    if (!params) return mfail(h, QW_E_ARG, "params is NULL");
    const hipError_t e = hipMemcpyAsync(params, at<float>(h, h->p.P), 4 * (size_t)h->p.s.n_nets * h->p.np,
                                        hipMemcpyDeviceToDevice, as_stream(hip_stream));
    if (e != hipSuccess) return mhip(h, e, "get params");
    return QW_OK;
}

int qw_mlp_forward(qw_mlp h, const float* x, int32_t B, float* y, void* hip_stream)
{
    int rc = check_batch(h, x, B);
    if (rc != QW_OK) return rc;
    if (!y) return mfail(h, QW_E_ARG, "y is NULL");
    hipStream_t s = as_stream(hip_stream);
    const Plan& p = h->p;
    hipError_t e = forward(h, ws_act(h), x, nullptr, B, s);
    // compact [net][B][n_out] from the padded [net][Mpad][16]
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(y, sizeof(float) * p.s.n_out, at<float>(h, p.Y), sizeof(float) * kInPad,
                             sizeof(float) * p.s.n_out, (size_t)B, hipMemcpyDeviceToDevice, s);
    for (int k = 1; k < p.s.n_nets && e == hipSuccess; ++k)
        e = hipMemcpy2DAsync(y + (size_t)k * B * p.s.n_out, sizeof(float) * p.s.n_out,
                             at<float>(h, p.Y) + (size_t)k * p.Mpad * kInPad, sizeof(float) * kInPad,
                             sizeof(float) * p.s.n_out, (size_t)B, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mhip(h, e, "forward");
    return QW_OK;
}

int qw_mlp_predict(qw_mlp h, const float* x, int32_t B, float* mean, float* spread, void* hip_stream)
{
    int rc = check_batch(h, x, B);
    if (rc != QW_OK) return rc;
    if (!mean || !spread) return mfail(h, QW_E_ARG, "mean or spread is NULL");
    hipStream_t s = as_stream(hip_stream);
    const Plan& p = h->p;
    hipError_t e = forward(h, ws_act(h), x, nullptr, B, s);
    if (e == hipSuccess)
        e = qwm::launch_ensemble(at<float>(h, p.Y), (long long)p.Mpad * kInPad, kInPad, B, p.s.n_out, p.s.n_nets,
                                 at<float>(h, p.oshift), at<float>(h, p.oscale), at<float>(h, p.swt), mean, spread,
                                 s);
    if (e != hipSuccess) return mhip(h, e, "predict");
    return QW_OK;
}

int qw_mlp_predict_static(qw_mlp h, const float* x, int32_t B, float* mean, float* spread, void* hip_stream)
{
    int rc = check_batch(h, x, B);
    if (rc != QW_OK) return rc;
    if (!mean || !spread) return mfail(h, QW_E_ARG, "mean or spread is NULL");
    if (B > QW_MLP_STATIC_MAX_BATCH)
        return mfail(h, QW_E_SIZE, "batch %d exceeds the static path's maximum of %d", B, QW_MLP_STATIC_MAX_BATCH);
    const Plan& p = h->p;
    const int M = round64(B);
    const ActLayout L = act_layout(p, M);
    if (L.total > kScratchBytes)
        return mfail(h, QW_E_SIZE, "a batch of %d of this network needs %zu bytes of scratch, the static array has %zu",
                     B, L.total, kScratchBytes);
    char* base = static_cast<char*>(scratch_of(h->device));
    if (!base) return mfail(h, QW_E_STATE, "static scratch of device %d was not set up", h->device);
    // every region is written before it is read (inputs zero-padded by the
    // input kernel, activations and outputs by the products): nothing to clear
    const Act a{reinterpret_cast<__bf16*>(base + L.xb), reinterpret_cast<__bf16*>(base + L.xt),
                reinterpret_cast<__bf16*>(base + L.hh), reinterpret_cast<float*>(base + L.y), M};
    hipStream_t s = as_stream(hip_stream);
    hipError_t e = forward(h, a, x, nullptr, B, s);
    if (e == hipSuccess)
        e = qwm::launch_ensemble(a.Y, (long long)M * kInPad, kInPad, B, p.s.n_out, p.s.n_nets, at<float>(h, p.oshift),
                                 at<float>(h, p.oscale), at<float>(h, p.swt), mean, spread, s);
    if (e != hipSuccess) return mhip(h, e, "predict (static scratch)");
    return QW_OK;
}

int qw_mlp_gradients(qw_mlp h, const float* x, const float* t, int32_t B, float* grads, float* loss,
                     void* hip_stream)
{
    int rc = check_batch(h, x, B);
    if (rc != QW_OK) return rc;
    if (!t) return mfail(h, QW_E_ARG, "t is NULL");
    hipStream_t s = as_stream(hip_stream);
    const Plan& p = h->p;
    hipError_t e = forward(h, ws_act(h), x, t, B, s);
    if (e == hipSuccess) e = backward(h, B, s);
    if (e == hipSuccess && grads)
        e = hipMemcpyAsync(grads, at<float>(h, p.G), 4 * (size_t)p.s.n_nets * p.np, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && loss)
        e = hipMemcpyAsync(loss, at<float>(h, p.loss), 4 * (size_t)p.s.n_nets, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mhip(h, e, "gradients");
    return QW_OK;
}

int qw_mlp_train_step(qw_mlp h, const float* x, const float* t, int32_t B, float lr, float* loss, void* hip_stream)
{
    int rc = check_batch(h, x, B);
    if (rc != QW_OK) return rc;
    if (!t) return mfail(h, QW_E_ARG, "t is NULL");
    if (!std::isfinite(lr) || lr < 0) return mfail(h, QW_E_ARG, "learning rate must be finite and >= 0");
    hipStream_t s = as_stream(hip_stream);
    const Plan& p = h->p;
    hipError_t e = forward(h, ws_act(h), x, t, B, s);
    if (e == hipSuccess) e = backward(h, B, s);
    h->t += 1;
    if (e == hipSuccess) e = qwm::launch_adam(adam_args(h, 1, lr), p.s.n_nets, s);
    if (e == hipSuccess && loss)
        e = hipMemcpyAsync(loss, at<float>(h, p.loss), 4 * (size_t)p.s.n_nets, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mhip(h, e, "train step");
    return QW_OK;
}

int qw_gemm_bf16_nt(const void* A, int32_t lda, const void* B, int32_t ldb, float* C, int32_t ldc, int32_t M,
                    int32_t N, int32_t K, void* hip_stream)
{
    if (!A || !B || !C) return mfail(nullptr, QW_E_ARG, "A, B or C is NULL");
    if (M < 1 || N < 1 || K < 16 || K % 16 != 0) return mfail(nullptr, QW_E_SIZE, "need M, N >= 1 and K a multiple of 16");
    if (lda < K || ldb < K || lda % 8 != 0 || ldb % 8 != 0 || ldc < N)
        return mfail(nullptr, QW_E_ARG, "leading dimensions: lda, ldb >= K and multiples of 8, ldc >= N");
    if (reinterpret_cast<uintptr_t>(A) % 16 != 0 || reinterpret_cast<uintptr_t>(B) % 16 != 0)
        return mfail(nullptr, QW_E_ARG, "A and B must be 16-byte aligned");
    qwm::GemmArgs g{};
    g.A = static_cast<const __bf16*>(A);
    g.lda = lda;
    g.B = static_cast<const __bf16*>(B);
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.Mpad = round64(M);
    g.Cf = C;
    g.ldcf = ldc;
    const hipError_t e = qwm::launch_gemm(qwm::EPI_F32, g, 1, N, as_stream(hip_stream));
    if (e != hipSuccess) return mfail(nullptr, QW_E_DEVICE, "gemm: %s", hipGetErrorString(e));
    return QW_OK;
}

const char* qw_mlp_last_error(qw_mlp h)
{
    if (!h) return g_mlp_error.c_str();
    return h->err.c_str();
}

void qw_mlp_destroy(qw_mlp h) { delete h; }

}  // extern "C"
