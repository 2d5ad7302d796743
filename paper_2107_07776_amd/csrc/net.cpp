// Learned pressure-guess network: parameters, activations and the C ABI
// (create, forward, backward, MSE, Adam, parameter access).
//
// Four 3x3x3 circular convolutions 6 -> 32 -> 32 -> 32 -> 2 with ReLU between
// them; bf16 weights and activations, FP32 accumulation, FP32 master
// parameters in the flat order [W0, b0, W1, b1, W2, b2, W3, b3] with each W
// as [out][in][dz][dy][dx].
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using trbdg::Error;
using trbdg::NetGeo;

namespace {
constexpr int NET_IN = 6, NET_OUT = 2;   // network input channels, outputs per voxel
}

struct tbdg_net {
    struct Layer {
        int cin_real, cout_real, cin, cout;   // cin, cout: padded to the kernel shapes
        int64_t w_off, b_off;
        int S;                                // forward slots
        uint16_t* Wp = nullptr;
        float* bias = nullptr;
        int cin2 = 0, Sb = 0;                 // input-gradient convolution
        uint16_t* Wt = nullptr;
    };
    int C = 32;
    hipStream_t stream = nullptr;
    std::string last_error;
    int64_t np = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    int64_t t = 0;
    Layer L[4];
    NetGeo geo{0, 0, 0, 0, 0};
    int64_t cap = 0;                          // activation capacity in voxels
    uint16_t* act[4] = {nullptr, nullptr, nullptr, nullptr};
    uint16_t* dbuf[2] = {nullptr, nullptr};
    uint16_t* d4 = nullptr;
    float* wpart = nullptr;
    int64_t wpart_cap = 0;
    double* lpart = nullptr;
    double* host = nullptr;
    bool packed = false;
    bool have_forward = false;
    std::vector<void*> allocs;
};

namespace {

template <typename T>
T* nalloc(tbdg_net* n, int64_t count) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, sizeof(T) * (size_t)(count > 0 ? count : 1));
    if (e != hipSuccess) throw Error(TBDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    n->allocs.push_back(p);
    return static_cast<T*>(p);
}

void nfree(tbdg_net* n, void* p) {
    if (!p) return;
    for (auto& a : n->allocs)
        if (a == p) {
            (void)hipFree(p);
            a = nullptr;
        }
}

template <class F>
tbdg_status guarded(tbdg_net* n, F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        if (n) n->last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        if (n) n->last_error = "host allocation failed";
        return TBDG_ENOMEM;
    } catch (const std::exception& e) {
        if (n) n->last_error = e.what();
        return TBDG_EINVAL;
    }
}

void require(bool ok, const char* msg) {
    if (!ok) throw Error(TBDG_EINVAL, msg);
}

uint64_t splitmix64_next(uint64_t& s) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void pack_all(tbdg_net* n) {
    for (int l = 0; l < 4; ++l) {
        auto& Y = n->L[l];
        trbdg::net_pack_fwd(n->stream, n->theta, Y.w_off, Y.cout_real, Y.cin_real, Y.cin, Y.cout, Y.S, Y.Wp);
        trbdg::net_copy_bias(n->stream, n->theta, Y.b_off, Y.cout_real, Y.bias);
        if (l > 0)
            trbdg::net_pack_bwd(n->stream, n->theta, Y.w_off, Y.cout_real, Y.cin_real, Y.cin2, Y.Sb, Y.Wt);
    }
    n->packed = true;
}

void ensure_capacity(tbdg_net* n, int64_t vox) {
    if (vox <= n->cap) return;
    for (auto& a : n->act) nfree(n, a);
    for (auto& d : n->dbuf) nfree(n, d);
    nfree(n, n->d4);
    n->act[0] = nalloc<uint16_t>(n, vox * 8);
    for (int l = 1; l < 4; ++l) n->act[l] = nalloc<uint16_t>(n, vox * n->C);
    n->dbuf[0] = nalloc<uint16_t>(n, vox * n->C);
    n->dbuf[1] = nalloc<uint16_t>(n, vox * n->C);
    n->d4 = nalloc<uint16_t>(n, vox * 8);
    n->cap = vox;
}

void wgrad(tbdg_net* n, int l, const uint16_t* X, const uint16_t* dY, int dys) {
    auto& Y = n->L[l];
    const NetGeo& g = n->geo;
    const int cout = Y.cout_real;   // gradient rows are the real outputs
    const int rows = g.B * g.ny * g.nz;
    int rpb = rows / 256;
    if (rpb < 1) rpb = 1;
    const int G = (rows + rpb - 1) / rpb;
    const int64_t npl = (int64_t)cout * Y.cin * 27 + cout;
    if ((int64_t)G * npl > n->wpart_cap) {
        nfree(n, n->wpart);
        n->wpart_cap = (int64_t)G * npl;
        n->wpart = nalloc<float>(n, n->wpart_cap);
    }
    trbdg::net_wgrad(n->stream, g, Y.cin, cout, dys, X, dY, n->wpart, rpb);
    trbdg::net_wgrad_reduce(n->stream, n->wpart, G, cout, Y.cin, Y.cin_real, n->grad, Y.w_off, Y.b_off);
}

}  // namespace

extern "C" {

tbdg_status tbdg_net_create(int channels, uint64_t seed, void* hip_stream, tbdg_net** out) {
    if (!out) return TBDG_EINVAL;
    *out = nullptr;
    tbdg_net* n = new (std::nothrow) tbdg_net();
    if (!n) return TBDG_ENOMEM;
    const tbdg_status st = guarded(n, [&]() {
        if (channels != 32) throw Error(TBDG_EUNSUPPORTED, "the network is built with 32 channels");
        n->C = channels;
        n->stream = static_cast<hipStream_t>(hip_stream);
        const int cin_real[4] = {NET_IN, 32, 32, 32}, cout_real[4] = {32, 32, 32, NET_OUT};
        const int cin[4] = {8, 32, 32, 32}, cout[4] = {32, 32, 32, 16};
        int64_t off = 0;
        for (int l = 0; l < 4; ++l) {
            auto& Y = n->L[l];
            Y.cin_real = cin_real[l];
            Y.cout_real = cout_real[l];
            Y.cin = cin[l];
            Y.cout = cout[l];
            Y.w_off = off;
            off += (int64_t)cout_real[l] * cin_real[l] * 27;
            Y.b_off = off;
            off += cout_real[l];
            Y.S = (27 * (cin[l] / 8) + 3) / 4 * 4;
            Y.Wp = nalloc<uint16_t>(n, (int64_t)Y.S * Y.cout * 8);
            Y.bias = nalloc<float>(n, 32);
            if (l > 0) {
                Y.cin2 = cout_real[l] < 8 ? 8 : cout_real[l];
                Y.Sb = (27 * (Y.cin2 / 8) + 3) / 4 * 4;
                Y.Wt = nalloc<uint16_t>(n, (int64_t)Y.Sb * Y.cin_real * 8);
            }
        }
        n->np = off;
        n->theta = nalloc<float>(n, n->np);
        n->grad = nalloc<float>(n, n->np);
        n->m = nalloc<float>(n, n->np);
        n->v = nalloc<float>(n, n->np);
        n->lpart = nalloc<double>(n, 1024);
        void* h = nullptr;
        TBDG_HIP(hipHostMalloc(&h, sizeof(double) * 1024, hipHostMallocDefault));
        n->host = static_cast<double*>(h);
        // He-uniform weights U(-a, a), a = sqrt(6 / fan_in), from SplitMix64,
        // for the hidden layers; the output layer and every bias start at
        // zero (the network starts from a zero correction)
        std::vector<float> th(n->np, 0.0f);
        uint64_t s = seed;
        for (int l = 0; l < 3; ++l) {
            const auto& Y = n->L[l];
            const double a = std::sqrt(6.0 / (27.0 * Y.cin_real));
            for (int64_t i = 0; i < (int64_t)Y.cout_real * Y.cin_real * 27; ++i) {
                const double u = (double)(splitmix64_next(s) >> 11) * 0x1.0p-53;
                th[Y.w_off + i] = (float)((2.0 * u - 1.0) * a);
            }
        }
        TBDG_HIP(hipMemcpyAsync(n->theta, th.data(), sizeof(float) * n->np, hipMemcpyHostToDevice, n->stream));
        TBDG_HIP(hipMemsetAsync(n->grad, 0, sizeof(float) * n->np, n->stream));
        TBDG_HIP(hipMemsetAsync(n->m, 0, sizeof(float) * n->np, n->stream));
        TBDG_HIP(hipMemsetAsync(n->v, 0, sizeof(float) * n->np, n->stream));
        TBDG_HIP(hipStreamSynchronize(n->stream));
        return TBDG_OK;
    });
    if (st != TBDG_OK) {
        for (void* p : n->allocs)
            if (p) (void)hipFree(p);
        if (n->host) (void)hipHostFree(n->host);
        delete n;
        return st;
    }
    *out = n;
    return TBDG_OK;
}

void tbdg_net_destroy(tbdg_net* n) {
    if (!n) return;
    (void)hipStreamSynchronize(n->stream);
    for (void* p : n->allocs)
        if (p) (void)hipFree(p);
    if (n->host) (void)hipHostFree(n->host);
    delete n;
}

const char* tbdg_net_last_error(const tbdg_net* n) { return n ? n->last_error.c_str() : "null network"; }

tbdg_status tbdg_net_num_params(const tbdg_net* n, int64_t* np) {
    if (!n || !np) return TBDG_EINVAL;
    *np = n->np;
    return TBDG_OK;
}

tbdg_status tbdg_net_set_params(tbdg_net* n, const float* theta) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(theta != nullptr, "null pointer");
        TBDG_HIP(hipMemcpyAsync(n->theta, theta, sizeof(float) * n->np, hipMemcpyDeviceToDevice, n->stream));
        TBDG_HIP(hipMemsetAsync(n->m, 0, sizeof(float) * n->np, n->stream));
        TBDG_HIP(hipMemsetAsync(n->v, 0, sizeof(float) * n->np, n->stream));
        n->t = 0;
        n->packed = false;
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_get_params(tbdg_net* n, float* theta) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(theta != nullptr, "null pointer");
        TBDG_HIP(hipMemcpyAsync(theta, n->theta, sizeof(float) * n->np, hipMemcpyDeviceToDevice, n->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_get_grads(tbdg_net* n, float* g) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(g != nullptr, "null pointer");
        TBDG_HIP(hipMemcpyAsync(g, n->grad, sizeof(float) * n->np, hipMemcpyDeviceToDevice, n->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_zero_grad(tbdg_net* n) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        TBDG_HIP(hipMemsetAsync(n->grad, 0, sizeof(float) * n->np, n->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_forward(tbdg_net* n, const float* x, float* y, int B, int nx, int ny, int nz) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(x && y, "null pointer");
        require(B >= 1 && nx >= 1 && ny >= 1 && nz >= 1, "empty batch or grid");
        const int64_t nvox = (int64_t)nx * ny * nz;
        require(nvox * B < (int64_t)1 << 31, "batch too large");
        if ((size_t)nx * (32 * 4 + 9 * 32 * 2) > 65536)
            throw Error(TBDG_EUNSUPPORTED, "grid rows longer than 93 voxels are not supported");
        n->geo = NetGeo{nx, ny, nz, (int)nvox, B};
        ensure_capacity(n, nvox * B);
        if (!n->packed) pack_all(n);
        const NetGeo& g = n->geo;
        trbdg::net_to_channel_last(n->stream, x, B, NET_IN, (int)nvox, 8, n->act[0]);
        trbdg::net_conv(n->stream, g, 8, 32, 0, n->act[0], n->L[0].Wp, n->L[0].bias, n->act[1], nullptr, nullptr);
        trbdg::net_conv(n->stream, g, 32, 32, 0, n->act[1], n->L[1].Wp, n->L[1].bias, n->act[2], nullptr, nullptr);
        trbdg::net_conv(n->stream, g, 32, 32, 0, n->act[2], n->L[2].Wp, n->L[2].bias, n->act[3], nullptr, nullptr);
        trbdg::net_conv(n->stream, g, 32, 16, 1, n->act[3], n->L[3].Wp, n->L[3].bias, nullptr, y, nullptr,
                        NET_OUT);
        n->have_forward = true;
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_backward(tbdg_net* n, const float* dy) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(dy != nullptr, "null pointer");
        if (!n->have_forward) throw Error(TBDG_EINVAL, "backward needs a preceding forward");
        if (!n->packed) pack_all(n);
        const NetGeo& g = n->geo;
        trbdg::net_to_channel_last(n->stream, dy, g.B, NET_OUT, g.nvox, 8, n->d4);
        wgrad(n, 3, n->act[3], n->d4, 8);
        trbdg::net_conv(n->stream, g, 8, 32, 2, n->d4, n->L[3].Wt, nullptr, n->dbuf[0], nullptr, n->act[3]);
        wgrad(n, 2, n->act[2], n->dbuf[0], 32);
        trbdg::net_conv(n->stream, g, 32, 32, 2, n->dbuf[0], n->L[2].Wt, nullptr, n->dbuf[1], nullptr, n->act[2]);
        wgrad(n, 1, n->act[1], n->dbuf[1], 32);
        trbdg::net_conv(n->stream, g, 32, 32, 2, n->dbuf[1], n->L[1].Wt, nullptr, n->dbuf[0], nullptr, n->act[1]);
        wgrad(n, 0, n->act[0], n->dbuf[0], 32);
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_mse(tbdg_net* n, const float* yhat, const float* target, int64_t count, float* dy,
                         double* loss) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(yhat && target && dy && count > 0, "null pointer or empty");
        const int G = trbdg::net_mse(n->stream, yhat, target, count, dy, n->lpart);
        if (loss) {
            TBDG_HIP(hipMemcpyAsync(n->host, n->lpart, sizeof(double) * G, hipMemcpyDeviceToHost, n->stream));
            TBDG_HIP(hipStreamSynchronize(n->stream));
            double s = 0.0;
            for (int i = 0; i < G; ++i) s += n->host[i];
            *loss = s / (double)count;
        }
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_quad_loss(tbdg_net* n, const float* yhat, const float* gram, int64_t count, int B,
                               float* dy, double* loss) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(yhat && gram && dy && count > 0 && B >= 1, "null pointer or empty");
        const int G = trbdg::net_quad_loss(n->stream, yhat, gram, count, B, dy, n->lpart);
        if (loss) {
            TBDG_HIP(hipMemcpyAsync(n->host, n->lpart, sizeof(double) * G, hipMemcpyDeviceToHost, n->stream));
            TBDG_HIP(hipStreamSynchronize(n->stream));
            double s = 0.0;
            for (int i = 0; i < G; ++i) s += n->host[i];
            *loss = s / ((double)count * B);
        }
        return TBDG_OK;
    });
}

tbdg_status tbdg_net_adam_step(tbdg_net* n, float lr, float beta1, float beta2, float eps) {
    if (!n) return TBDG_EINVAL;
    return guarded(n, [&]() {
        require(lr > 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f,
                "invalid Adam parameters");
        n->t += 1;
        const float c1 = (float)(1.0 - std::pow((double)beta1, (double)n->t));
        const float c2 = (float)(1.0 - std::pow((double)beta2, (double)n->t));
        trbdg::net_adam(n->stream, n->np, n->theta, n->grad, n->m, n->v, lr, beta1, beta2, eps, c1, c2);
        n->packed = false;
        return TBDG_OK;
    });
}

}  // extern "C"

namespace trbdg {

hipStream_t net_stream(const tbdg_net* net) { return net->stream; }

void net_infer(tbdg_net* net, const float* x, float* y, int nx, int ny, int nz) {
    const tbdg_status st = tbdg_net_forward(net, x, y, 1, nx, ny, nz);
    if (st != TBDG_OK) throw Error(st, std::string("guess network: ") + net->last_error);
}

}  // namespace trbdg
