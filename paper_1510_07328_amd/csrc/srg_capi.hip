// C ABI of the convolutional surrogate: context and workspace, forward,
// backward, loss, Adam, a training step, the mass-residual indicator and the
// hybrid advance of a tube batch (surrogate jump with the lattice BGK run as
// fallback).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "srg.h"

namespace lbm {
void set_last_error(const std::string &msg);
hipStream_t batch_stream(const lbm_batch_s *b);
void batch_shape(const lbm_batch_s *b, int *ntubes, int *nx);
hipError_t batch_device_schedule(lbm_batch_s *b, int nsteps);
hipError_t batch_profiles_dev(lbm_batch_s *b, float *prof_dev, const unsigned char *skip);
hipError_t batch_set_profiles_dev(lbm_batch_s *b, const unsigned char *mask, const float *prof_dev);
hipError_t batch_commit_dev(lbm_batch_s *b, unsigned char *lazy, float *pin, const float *pout);
hipError_t clear_bytes(unsigned char *p, int n, hipStream_t s);
hipError_t batch_decide_dev(lbm_batch_s *b, const float *resid_dev, float tol, int *count_dev);
hipError_t batch_rounds_dev(lbm_batch_s *b);
}

namespace srg {
hipError_t l1_fwd(const float *nu, const float *tau, const __bf16 *W1, const float *b1, __bf16 *z1, __bf16 *a1, int B,
                  int L, hipStream_t s);
hipError_t hidden(bool dgrad, const __bf16 *in, const __bf16 *Wop, const float *bias, const __bf16 *zprev,
                  __bf16 *out_z, __bf16 *out_a, int B, int L, int d, hipStream_t s);
hipError_t hidden_wgrad(const __bf16 *dz, const __bf16 *a, float *part, float *partb, int G, int B, int L, int d,
                        hipStream_t s);
hipError_t l4_fwd(const __bf16 *a3, const __bf16 *W4, const float *b4, const float *nu, float *out, int B, int L,
                  hipStream_t s);
hipError_t fwd_fused(const float *nu, const float *tau, const __bf16 *W1, const float *b1, const __bf16 *W2,
                     const float *b2, const __bf16 *W3, const float *b3, const __bf16 *W4, const float *b4, float *out,
                     int B, int L, hipStream_t s);
int fused_max_length();
hipError_t l4_dgrad(const float *dout, const __bf16 *W4, const __bf16 *z3, __bf16 *dz3, int B, int L, hipStream_t s);
hipError_t l4_wgrad(const float *dout, const __bf16 *a3, float *part, int G, int B, int L, hipStream_t s);
hipError_t l1_wgrad(const __bf16 *dz1, const float *nu, const float *tau, float *part, int G, int B, int L,
                    hipStream_t s);
hipError_t reduce(const float *part, int G, int n, float *dst, hipStream_t s);
hipError_t loss(const float *out, const float *target, float *dout, float *stats, int B, int L, float lambda,
                hipStream_t s);
hipError_t mass_residual(const float *in, const float *out, float *resid, int B, int L, hipStream_t s);
hipError_t indicator(const float *in, const float *out, float *resid, int B, int L, hipStream_t s);
hipError_t adam(float *p, float *m, float *v, const float *g, int n, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t s);
hipError_t to_bf16(const float *src, __bf16 *dst, int n, hipStream_t s);
hipError_t transpose_bf16(const float *src, __bf16 *dst, hipStream_t s);
}  // namespace srg

namespace {

constexpr int CH = 64, KT = 5;
// flat parameter layout: W1 b1 W2 b2 W3 b3 W4 b4, each W [tap][co][ci]
constexpr int NW1 = KT * CH * 3, NW2 = KT * CH * CH, NW4 = KT * 2 * CH;
constexpr int OW1 = 0, OB1 = OW1 + NW1, OW2 = OB1 + CH, OB2 = OW2 + NW2, OW3 = OB2 + CH, OB3 = OW3 + NW2,
              OW4 = OB3 + CH, OB4 = OW4 + NW4, NPARAM = OB4 + 2;
constexpr int G = 256;  // workgroups of the weight-gradient reductions
constexpr int DIL[4] = {1, 3, 9, 27};
constexpr int NCOUNT = 1024;  // fallback counts kept on the device between read-backs

lbm_status sfail(lbm_status s, const std::string &m) {
    lbm::set_last_error(m);
    return s;
}
lbm_status shipf(hipError_t e, const char *what) {
    lbm::set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    return LBM_ERR_HIP;
}
size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct Carve {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count) {
        const size_t o = off;
        off = al(off + count * sizeof(T));
        return o;
    }
};

struct Offsets {
    size_t master, m, v, grad, w1b, w2b, w2t, w3b, w3t, w4b, act[6], dz[3], part, partb, part4, part1, dout, stats,
        resid, counts, prof_in, prof_out, lazy, total;
};

Offsets layout(int B, int L) {
    Carve c;
    Offsets o;
    o.master = c.take<float>(NPARAM);
    o.m = c.take<float>(NPARAM);
    o.v = c.take<float>(NPARAM);
    o.grad = c.take<float>(NPARAM);
    o.w1b = c.take<__bf16>(NW1);
    o.w2b = c.take<__bf16>(NW2);
    o.w2t = c.take<__bf16>(NW2);
    o.w3b = c.take<__bf16>(NW2);
    o.w3t = c.take<__bf16>(NW2);
    o.w4b = c.take<__bf16>(NW4);
    const size_t act = (size_t)B * L * CH;
    for (auto &a : o.act) a = c.take<__bf16>(act);
    for (auto &a : o.dz) a = c.take<__bf16>(act);
    o.part = c.take<float>((size_t)G * NW2);
    o.partb = c.take<float>((size_t)G * CH);
    o.part4 = c.take<float>((size_t)G * (NW4 + 2));
    o.part1 = c.take<float>((size_t)G * (NW1 + CH));
    o.dout = c.take<float>((size_t)B * 2 * L);
    o.stats = c.take<float>((size_t)B * 2);
    o.resid = c.take<float>((size_t)B);
    o.counts = c.take<int>(NCOUNT);
    o.prof_in = c.take<float>((size_t)B * 2 * L);
    o.prof_out = c.take<float>((size_t)B * 2 * L);
    o.lazy = c.take<unsigned char>((size_t)B);
    o.total = c.off;
    return o;
}

}  // namespace

struct srg_ctx_s {
    int maxB = 0, L = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    Offsets o{};
    int step = 0;
    int lastB = 0;
    const float *last_nu = nullptr, *last_tau = nullptr;
    template <typename T>
    T *at(size_t off) {
        return reinterpret_cast<T *>(ws + off);
    }
};

namespace {

hipError_t prepare_weights(srg_ctx_s *c) {
    const float *p = c->at<float>(c->o.master);
    hipError_t e = srg::to_bf16(p + OW1, c->at<__bf16>(c->o.w1b), NW1, c->stream);
    if (e == hipSuccess) e = srg::to_bf16(p + OW2, c->at<__bf16>(c->o.w2b), NW2, c->stream);
    if (e == hipSuccess) e = srg::transpose_bf16(p + OW2, c->at<__bf16>(c->o.w2t), c->stream);
    if (e == hipSuccess) e = srg::to_bf16(p + OW3, c->at<__bf16>(c->o.w3b), NW2, c->stream);
    if (e == hipSuccess) e = srg::transpose_bf16(p + OW3, c->at<__bf16>(c->o.w3t), c->stream);
    if (e == hipSuccess) e = srg::to_bf16(p + OW4, c->at<__bf16>(c->o.w4b), NW4, c->stream);
    return e;
}

// keep = true: layer by layer, the activations (and pre-activations z) kept for
// a backward pass; keep = false: inference, all layers in one kernel for lengths
// up to srg::fused_max_length() (the same result bit for bit, nothing kept),
// layer by layer without the z beyond
hipError_t forward(srg_ctx_s *c, const float *nu, const float *tau, int B, float *out, bool keep) {
    const int L = c->L;
    const float *p = c->at<float>(c->o.master);
    if (!keep && L <= srg::fused_max_length()) {
        c->lastB = 0;
        return srg::fwd_fused(nu, tau, c->at<__bf16>(c->o.w1b), p + OB1, c->at<__bf16>(c->o.w2b), p + OB2,
                              c->at<__bf16>(c->o.w3b), p + OB3, c->at<__bf16>(c->o.w4b), p + OB4, out, B, L, c->stream);
    }
    __bf16 *z1 = c->at<__bf16>(c->o.act[0]), *a1 = c->at<__bf16>(c->o.act[1]);
    __bf16 *z2 = c->at<__bf16>(c->o.act[2]), *a2 = c->at<__bf16>(c->o.act[3]);
    __bf16 *z3 = c->at<__bf16>(c->o.act[4]), *a3 = c->at<__bf16>(c->o.act[5]);
    if (!keep) z1 = z2 = z3 = nullptr;
    hipError_t e = srg::l1_fwd(nu, tau, c->at<__bf16>(c->o.w1b), p + OB1, z1, a1, B, L, c->stream);
    if (e == hipSuccess)
        e = srg::hidden(false, a1, c->at<__bf16>(c->o.w2b), p + OB2, nullptr, z2, a2, B, L, DIL[1], c->stream);
    if (e == hipSuccess)
        e = srg::hidden(false, a2, c->at<__bf16>(c->o.w3b), p + OB3, nullptr, z3, a3, B, L, DIL[2], c->stream);
    if (e == hipSuccess) e = srg::l4_fwd(a3, c->at<__bf16>(c->o.w4b), p + OB4, nu, out, B, L, c->stream);
    c->lastB = keep ? B : 0;
    c->last_nu = nu;
    c->last_tau = tau;
    return e;
}

hipError_t backward(srg_ctx_s *c, const float *dout, float *grad) {
    const int B = c->lastB, L = c->L;
    __bf16 *z1 = c->at<__bf16>(c->o.act[0]), *a1 = c->at<__bf16>(c->o.act[1]);
    __bf16 *z2 = c->at<__bf16>(c->o.act[2]), *a2 = c->at<__bf16>(c->o.act[3]);
    __bf16 *z3 = c->at<__bf16>(c->o.act[4]), *a3 = c->at<__bf16>(c->o.act[5]);
    __bf16 *dz3 = c->at<__bf16>(c->o.dz[2]), *dz2 = c->at<__bf16>(c->o.dz[1]), *dz1 = c->at<__bf16>(c->o.dz[0]);
    float *part = c->at<float>(c->o.part), *partb = c->at<float>(c->o.partb);
    float *part4 = c->at<float>(c->o.part4), *part1 = c->at<float>(c->o.part1);
    const int g = B < G ? B : G;
    hipError_t e = srg::l4_wgrad(dout, a3, part4, g, B, L, c->stream);
    if (e == hipSuccess) e = srg::reduce(part4, g, NW4 + 2, grad + OW4, c->stream);  // W4 then b4 (contiguous)
    if (e == hipSuccess) e = srg::l4_dgrad(dout, c->at<__bf16>(c->o.w4b), z3, dz3, B, L, c->stream);
    // layer 3: weights, then the data gradient into layer 2's dz
    if (e == hipSuccess) e = srg::hidden_wgrad(dz3, a2, part, partb, g, B, L, DIL[2], c->stream);
    if (e == hipSuccess) e = srg::reduce(part, g, NW2, grad + OW3, c->stream);
    if (e == hipSuccess) e = srg::reduce(partb, g, CH, grad + OB3, c->stream);
    if (e == hipSuccess)
        e = srg::hidden(true, dz3, c->at<__bf16>(c->o.w3t), nullptr, z2, dz2, nullptr, B, L, DIL[2], c->stream);
    // layer 2
    if (e == hipSuccess) e = srg::hidden_wgrad(dz2, a1, part, partb, g, B, L, DIL[1], c->stream);
    if (e == hipSuccess) e = srg::reduce(part, g, NW2, grad + OW2, c->stream);
    if (e == hipSuccess) e = srg::reduce(partb, g, CH, grad + OB2, c->stream);
    if (e == hipSuccess)
        e = srg::hidden(true, dz2, c->at<__bf16>(c->o.w2t), nullptr, z1, dz1, nullptr, B, L, DIL[1], c->stream);
    // layer 1 (weights only)
    if (e == hipSuccess) e = srg::l1_wgrad(dz1, c->last_nu, c->last_tau, part1, g, B, L, c->stream);
    if (e == hipSuccess) e = srg::reduce(part1, g, NW1 + CH, grad + OW1, c->stream);  // W1 then b1 (contiguous)
    return e;
}

lbm_status check_batch(const srg_ctx_s *c, int B) {
    if (!c) return sfail(LBM_ERR_ARG, "null context");
    if (B < 1 || B > c->maxB) return sfail(LBM_ERR_ARG, "batch must be in [1, max_batch]");
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status srg_param_count(int64_t *n) {
    if (!n) return sfail(LBM_ERR_ARG, "null argument");
    *n = NPARAM;
    return LBM_OK;
}

lbm_status srg_workspace_bytes(int max_batch, int length, size_t *bytes) {
    if (!bytes) return sfail(LBM_ERR_ARG, "null argument");
    if (max_batch < 1 || length < 128 || length % 128 || length > (1 << 20))
        return sfail(LBM_ERR_ARG, "need max_batch >= 1 and length a multiple of 128 (at most 2^20)");
    if ((double)max_batch * length > 1e9) return sfail(LBM_ERR_ARG, "max_batch * length too large");
    *bytes = layout(max_batch, length).total;
    return LBM_OK;
}

lbm_status srg_create(int max_batch, int length, void *workspace, size_t bytes, void *stream, srg_ctx *out) {
    if (!workspace || !out) return sfail(LBM_ERR_ARG, "null argument");
    *out = nullptr;
    size_t need = 0;
    lbm_status s = srg_workspace_bytes(max_batch, length, &need);
    if (s != LBM_OK) return s;
    if (bytes < need) return sfail(LBM_ERR_ARG, "workspace smaller than srg_workspace_bytes()");
    if ((uintptr_t)workspace % 256) return sfail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
    srg_ctx_s *c = new (std::nothrow) srg_ctx_s;
    if (!c) return sfail(LBM_ERR_ARG, "out of host memory");
    c->maxB = max_batch;
    c->L = length;
    c->stream = (hipStream_t)stream;
    c->ws = (char *)workspace;
    c->o = layout(max_batch, length);
    *out = c;
    return LBM_OK;
}

lbm_status srg_set_params(srg_ctx c, const float *params_dev) {
    if (!c || !params_dev) return sfail(LBM_ERR_ARG, "null argument");
    hipError_t e = hipMemcpyAsync(c->at<float>(c->o.master), params_dev, sizeof(float) * NPARAM,
                                  hipMemcpyDeviceToDevice, c->stream);
    // the Adam moments restart from zero
    if (e == hipSuccess) e = hipMemsetAsync(c->at<float>(c->o.m), 0, sizeof(float) * NPARAM, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->at<float>(c->o.v), 0, sizeof(float) * NPARAM, c->stream);
    if (e == hipSuccess) e = prepare_weights(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->step = 0;
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_set_params");
}

lbm_status srg_get_params(srg_ctx c, float *params_dev) {
    if (!c || !params_dev) return sfail(LBM_ERR_ARG, "null argument");
    hipError_t e = hipMemcpyAsync(params_dev, c->at<float>(c->o.master), sizeof(float) * NPARAM,
                                  hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_get_params");
}

lbm_status srg_forward(srg_ctx c, const float *nu_dev, const float *tau_dev, int batch, float *out_dev) {
    lbm_status s = check_batch(c, batch);
    if (s != LBM_OK) return s;
    if (!nu_dev || !tau_dev || !out_dev) return sfail(LBM_ERR_ARG, "null argument");
    hipError_t e = forward(c, nu_dev, tau_dev, batch, out_dev, true);
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_forward");
}

lbm_status srg_infer(srg_ctx c, const float *nu_dev, const float *tau_dev, int batch, float *out_dev) {
    lbm_status s = check_batch(c, batch);
    if (s != LBM_OK) return s;
    if (!nu_dev || !tau_dev || !out_dev) return sfail(LBM_ERR_ARG, "null argument");
    if (out_dev == nu_dev) return sfail(LBM_ERR_ARG, "out must not alias the input profiles");
    hipError_t e = forward(c, nu_dev, tau_dev, batch, out_dev, false);
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_infer");
}

lbm_status srg_backward(srg_ctx c, const float *dout_dev, float *grad_dev) {
    if (!c || !dout_dev || !grad_dev) return sfail(LBM_ERR_ARG, "null argument");
    if (c->lastB < 1) return sfail(LBM_ERR_STATE, "srg_backward needs a preceding srg_forward");
    hipError_t e = backward(c, dout_dev, grad_dev);
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_backward");
}

lbm_status srg_loss(srg_ctx c, const float *out_dev, const float *target_dev, int batch, float lambda_mass,
                    float *dout_dev, double *loss_host) {
    lbm_status s = check_batch(c, batch);
    if (s != LBM_OK) return s;
    if (!out_dev || !target_dev || !dout_dev) return sfail(LBM_ERR_ARG, "null argument");
    float *stats = c->at<float>(c->o.stats);
    hipError_t e = srg::loss(out_dev, target_dev, dout_dev, stats, batch, c->L, lambda_mass, c->stream);
    if (e == hipSuccess && loss_host) {
        std::vector<float> st(2 * batch);
        e = hipMemcpyAsync(st.data(), stats, sizeof(float) * 2 * batch, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) {
            double se = 0.0, sm = 0.0;
            for (int b = 0; b < batch; ++b) {
                se += st[2 * b];
                sm += (double)st[2 * b + 1] * st[2 * b + 1];
            }
            *loss_host = se / (2.0 * batch * c->L) + lambda_mass * sm / batch;
        }
    }
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_loss");
}

lbm_status srg_adam(srg_ctx c, const float *grad_dev, float lr, float b1, float b2, float eps) {
    if (!c || !grad_dev) return sfail(LBM_ERR_ARG, "null argument");
    if (!(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return sfail(LBM_ERR_ARG, "bad Adam hyper-parameters");
    c->step++;
    const float c1 = 1.0f - std::pow(b1, (float)c->step), c2 = 1.0f - std::pow(b2, (float)c->step);
    hipError_t e = srg::adam(c->at<float>(c->o.master), c->at<float>(c->o.m), c->at<float>(c->o.v), grad_dev, NPARAM,
                             lr, b1, b2, eps, c1, c2, c->stream);
    if (e == hipSuccess) e = prepare_weights(c);
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_adam");
}

lbm_status srg_train_step(srg_ctx c, const float *nu_dev, const float *tau_dev, const float *target_dev, int batch,
                          float lr, float lambda_mass, double *loss_host) {
    lbm_status s = check_batch(c, batch);
    if (s != LBM_OK) return s;
    if (!nu_dev || !tau_dev || !target_dev) return sfail(LBM_ERR_ARG, "null argument");
    float *out = c->at<float>(c->o.prof_out);
    hipError_t e = forward(c, nu_dev, tau_dev, batch, out, true);
    if (e != hipSuccess) return shipf(e, "srg_train_step forward");
    s = srg_loss(c, out, target_dev, batch, lambda_mass, c->at<float>(c->o.dout), loss_host);
    if (s != LBM_OK) return s;
    e = backward(c, c->at<float>(c->o.dout), c->at<float>(c->o.grad));
    if (e != hipSuccess) return shipf(e, "srg_train_step backward");
    return srg_adam(c, c->at<float>(c->o.grad), lr, 0.9f, 0.999f, 1e-8f);
}

lbm_status srg_mass_residual(srg_ctx c, const float *nu_in_dev, const float *nu_out_dev, int batch,
                             float *resid_dev) {
    lbm_status s = check_batch(c, batch);
    if (s != LBM_OK) return s;
    if (!nu_in_dev || !nu_out_dev || !resid_dev) return sfail(LBM_ERR_ARG, "null argument");
    hipError_t e = srg::mass_residual(nu_in_dev, nu_out_dev, resid_dev, batch, c->L, c->stream);
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_mass_residual");
}

lbm_status srg_hybrid_advance(srg_ctx c, lbm_batch b, const float *tau_dev, int ntubes, int jumps, int jump_steps,
                              float mass_tol, int *fallback_host) {
    lbm_status s = check_batch(c, ntubes);
    if (s != LBM_OK) return s;
    if (!b || !tau_dev || jumps < 0 || jump_steps < 1 || jump_steps > 0x3fffffff)
        return sfail(LBM_ERR_ARG, "bad hybrid arguments");
    int bt = 0, bnx = 0;
    lbm::batch_shape(b, &bt, &bnx);
    if (bt != ntubes) return sfail(LBM_ERR_ARG, "ntubes differs from the batch's tube count");
    if (bnx != c->L) return sfail(LBM_ERR_UNSUPPORTED, "tubes must all have the context's length");
    if (lbm::batch_stream(b) != c->stream) return sfail(LBM_ERR_ARG, "batch and surrogate must share one stream");
    if (jumps == 0) return LBM_OK;
    float *pin = c->at<float>(c->o.prof_in), *pout = c->at<float>(c->o.prof_out), *resid = c->at<float>(c->o.resid);
    int *counts = c->at<int>(c->o.counts);
    unsigned char *lazy = c->at<unsigned char>(c->o.lazy);
    hipError_t e = lbm::batch_device_schedule(b, jump_steps);
    if (e == hipSuccess) e = lbm::clear_bytes(lazy, ntubes, c->stream);
    if (e != hipSuccess) return shipf(e, "srg_hybrid_advance schedule");
    // Every jump is queued without waiting: the decision, the state updates and
    // the masked lattice advance all read the indicators on the device.  A tube
    // whose jump was accepted keeps the prediction as its state (pin, flag
    // lazy): the next jump starts from it as it is, and its populations are set
    // to f_eq of it only when a later jump falls back to the lattice, or at the
    // end.
    for (int j = 0; j < jumps; ++j) {
        e = lbm::batch_profiles_dev(b, pin, lazy);
        if (e == hipSuccess) e = forward(c, pin, tau_dev, ntubes, pout, false);
        if (e == hipSuccess) e = srg::indicator(pin, pout, resid, ntubes, c->L, c->stream);
        // the decision, the step counts and the list of the rejected tubes' tiles
        if (e == hipSuccess) e = lbm::batch_decide_dev(b, resid, mass_tol, counts + j % NCOUNT);
        if (e == hipSuccess) e = lbm::batch_commit_dev(b, lazy, pin, pout);
        if (e == hipSuccess) e = lbm::batch_rounds_dev(b);
        if (e == hipSuccess && j + 1 == jumps) e = lbm::batch_set_profiles_dev(b, lazy, pin);
        // read the counts back when the ring is full and at the end
        const bool flush = fallback_host && ((j + 1) % NCOUNT == 0 || j + 1 == jumps);
        if (e == hipSuccess && flush) {
            const int first = j / NCOUNT * NCOUNT;
            e = hipMemcpyAsync(fallback_host + first, counts, sizeof(int) * (j + 1 - first), hipMemcpyDeviceToHost,
                               c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        }
        if (e != hipSuccess) return shipf(e, "srg_hybrid_advance");
    }
    return LBM_OK;
}

lbm_status srg_free(srg_ctx c) {
    if (!c) return LBM_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    delete c;
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_free");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Inference without a context or workspace (srg_infer_noalloc).  Its only
// scratch is the bfloat16 copy of the four weight tensors, held in a static
// device array (one copy per GPU, for the life of the process); the biases are
// read from the caller's float32 parameters directly.  Host code never passes
// the array's name to a kernel or a copy: it asks the runtime for the array's
// address on each device once and uses that address.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t align256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t SW1 = 0, SW2 = SW1 + align256(NW1 * sizeof(__bf16)), SW3 = SW2 + align256(NW2 * sizeof(__bf16)),
                 SW4 = SW3 + align256(NW2 * sizeof(__bf16)), SCRATCH_BYTES = SW4 + align256(NW4 * sizeof(__bf16));
}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {
struct ScratchAddress {
    static constexpr int kMaxDevices = 64;
    std::mutex m;
    unsigned char *ptr[kMaxDevices] = {};
    // device address of `scratch` on the current device, looked up once per device
    hipError_t get(unsigned char **out) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
        std::lock_guard<std::mutex> lock(m);
        if (!ptr[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!p) return hipErrorInvalidSymbol;
            ptr[dev] = static_cast<unsigned char *>(p);
        }
        *out = ptr[dev];
        return hipSuccess;
    }
};
ScratchAddress g_scratch;
}  // namespace

extern "C" lbm_status srg_infer_noalloc(const float *params_dev, const float *prof_dev, const float *tau_dev,
                                        int batch, int length, float *out_dev, void *stream) {
    if (!params_dev || !prof_dev || !tau_dev || !out_dev) return sfail(LBM_ERR_ARG, "null argument");
    if (batch < 1) return sfail(LBM_ERR_ARG, "batch must be >= 1");
    if (length < 128 || length % 128 || length > srg::fused_max_length())
        return sfail(LBM_ERR_ARG, "srg_infer_noalloc: length must be a multiple of 128 in [128, " +
                                      std::to_string(srg::fused_max_length()) +
                                      "] (longer profiles need activation buffers: use srg_infer)");
    if (out_dev == prof_dev) return sfail(LBM_ERR_ARG, "out must not alias the input profiles");
    unsigned char *base = nullptr;
    hipError_t e = g_scratch.get(&base);
    if (e != hipSuccess) return shipf(e, "srg_infer_noalloc: scratch address");
    const hipStream_t s = (hipStream_t)stream;
    __bf16 *w1 = reinterpret_cast<__bf16 *>(base + SW1), *w2 = reinterpret_cast<__bf16 *>(base + SW2);
    __bf16 *w3 = reinterpret_cast<__bf16 *>(base + SW3), *w4 = reinterpret_cast<__bf16 *>(base + SW4);
    e = srg::to_bf16(params_dev + OW1, w1, NW1, s);
    if (e == hipSuccess) e = srg::to_bf16(params_dev + OW2, w2, NW2, s);
    if (e == hipSuccess) e = srg::to_bf16(params_dev + OW3, w3, NW2, s);
    if (e == hipSuccess) e = srg::to_bf16(params_dev + OW4, w4, NW4, s);
    if (e == hipSuccess)
        e = srg::fwd_fused(prof_dev, tau_dev, w1, params_dev + OB1, w2, params_dev + OB2, w3, params_dev + OB3, w4,
                           params_dev + OB4, out_dev, batch, length, s);
    return e == hipSuccess ? LBM_OK : shipf(e, "srg_infer_noalloc");
}
