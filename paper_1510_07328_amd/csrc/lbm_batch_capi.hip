// C ABI of the batched tube sweep: validation, workspace carving, the tile
// schedule, graph capture of a whole sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "lbm_batch.h"
#include "lbm_internal.h"

namespace lbm {
hipError_t batch_round(int fp64, void *b0, void *b1, const BatchTube *tubes, const BatchTile *tiles, const int *list,
                       int ntiles, int round, int H, int W, int block, const Model &m, double rho_ref, hipStream_t s);
hipError_t batch_decide_list(const float *resid, int ntubes, float tol, int nsteps, unsigned char *mask,
                             BatchTube *tubes, const BatchTile *tiles, int ntiles, int *list, int *count,
                             hipStream_t s);
hipError_t batch_set_steps(BatchTube *tubes, int ntubes, const int *steps, hipStream_t s);
hipError_t batch_flip(BatchTube *tubes, int ntubes, int H, hipStream_t s);
hipError_t batch_init(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes, const Model &m,
                      double rho_ref, hipStream_t s);
hipError_t batch_set_eq(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes, const unsigned char *mask,
                        const double *n, const double *u, int64_t total_cells, const Model &m, double rho_ref,
                        hipStream_t s);
hipError_t batch_moments(int fp64, const void *b0, const void *b1, const BatchTube *tubes, int ntubes, double *n,
                         double *u, int *bad, int64_t total_cells, double rho_ref, hipStream_t s);
hipError_t batch_profiles(int fp64, const void *b0, const void *b1, const BatchTube *tubes, int ntubes, float *prof,
                          double rho_ref, hipStream_t s, const unsigned char *skip = nullptr);
hipError_t batch_commit(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes, const unsigned char *mask,
                        unsigned char *lazy, float *pin, const float *pout, const Model &m, double rho_ref,
                        hipStream_t s);
hipError_t batch_set_profiles(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes,
                              const unsigned char *mask, const float *prof, const Model &m, double rho_ref,
                              hipStream_t s);
void set_last_error(const std::string &msg);
}  // namespace lbm

using namespace lbm;

namespace {

lbm_status bfail(lbm_status s, const std::string &msg) {
    set_last_error(msg);
    return s;
}

lbm_status bhip(hipError_t e, const char *what) {
    set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    return LBM_ERR_HIP;
}

constexpr size_t kAlign = 256;
size_t al(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr int NY = 4, Q = 9;
constexpr int kMaxWindow = 512;  // columns of the largest LDS window (float32: 72 KB, float64: 147 KB)

struct BatchLayout {
    int64_t cells = 0;
    int max_tiles = 0;
    size_t elt = 0, buf = 0, off_tubes = 0, off_tiles_run = 0, off_steps_run = 0, off_tiles_adv = 0,
           off_steps_adv = 0, off_mask = 0, off_bad = 0, off_list = 0, total = 0;
    int S = 0, H = 0, block = 0;
};

lbm_status check(const lbm_tube *tubes, int ntubes, const lbm_batch_options *opt, Model *m, BatchLayout *lay) {
    if (!tubes || !opt || ntubes < 1) return bfail(LBM_ERR_ARG, "need at least one tube and options");
    if (opt->precision != LBM_FP32_DEV && opt->precision != LBM_FP64) return bfail(LBM_ERR_ARG, "bad precision");
    if (opt->weight == LBM_W_FD_LOCAL)
        return bfail(LBM_ERR_UNSUPPORTED, "the batched sweep takes one weight for all cells (no per-cell weights)");
    lbm_config cfg{};
    cfg.lattice = LBM_D2V9;
    cfg.nx = 8;
    cfg.ny = NY;
    cfg.nz = 1;
    cfg.weight = opt->weight;
    cfg.J2 = opt->J2;
    cfg.J4 = opt->J4;
    cfg.fugacity = opt->fugacity;
    cfg.order = opt->order;
    cfg.tau = 1.0;
    std::string err;
    lbm_status s = build_model(&cfg, m, &err);
    if (s != LBM_OK) return bfail(s, err);
    lay->elt = opt->precision == LBM_FP64 ? 8 : 4;
    const int wmax = kMaxWindow;
    lay->H = opt->halo > 0 ? opt->halo : 32;
    lay->S = opt->tile_cols > 0 ? opt->tile_cols : 512 - 2 * lay->H;
    lay->block = opt->block > 0 ? opt->block : 1024;
    if (lay->block % 64 || lay->block > 1024) return bfail(LBM_ERR_ARG, "block must be a multiple of 64, <= 1024");
    if (lay->S < 1 || lay->S + 2 * lay->H > wmax)
        return bfail(LBM_ERR_ARG, "tile_cols + 2 halo exceeds the LDS window of " + std::to_string(wmax) + " columns");
    int64_t cells = 0;
    int64_t tiles = 0;
    for (int t = 0; t < ntubes; ++t) {
        const lbm_tube &tb = tubes[t];
        if (tb.nx < 2) return bfail(LBM_ERR_ARG, "tube " + std::to_string(t) + ": nx < 2");
        if (!(tb.tau > 0.5) || !std::isfinite(tb.tau)) return bfail(LBM_ERR_ARG, "tube tau must be > 1/2");
        if (tb.steps < 0 || tb.steps > 0x3fffffff) return bfail(LBM_ERR_ARG, "tube steps out of range");
        if (!(tb.n_left > 0) || !(tb.n_right > 0)) return bfail(LBM_ERR_ARG, "tube densities must be > 0");
        cells += (int64_t)NY * tb.nx;
        tiles += (tb.nx + lay->S - 1) / lay->S;
    }
    if (tiles > 0x7fffffff) return bfail(LBM_ERR_ARG, "too many tiles");
    lay->cells = cells;
    lay->max_tiles = (int)tiles;
    lay->buf = al((size_t)Q * cells * lay->elt);
    lay->off_tubes = 2 * lay->buf;
    lay->off_tiles_run = lay->off_tubes + al(sizeof(BatchTube) * ntubes);
    lay->off_steps_run = lay->off_tiles_run + al(sizeof(BatchTile) * tiles);
    lay->off_tiles_adv = lay->off_steps_run + al(sizeof(int) * ntubes);
    lay->off_steps_adv = lay->off_tiles_adv + al(sizeof(BatchTile) * tiles);
    lay->off_mask = lay->off_steps_adv + al(sizeof(int) * ntubes);
    lay->off_bad = lay->off_mask + al((size_t)ntubes);
    lay->off_list = lay->off_bad + al(sizeof(int) * ntubes);
    lay->total = lay->off_list + al(sizeof(int) * (tiles + 1));
    return LBM_OK;
}

// Tiles of the tubes with steps > 0, ordered by rounds (descending), and the
// number of active tiles in each round.
void schedule(const std::vector<lbm_tube> &tubes, const std::vector<int> &steps, int S, int H,
              std::vector<BatchTile> *tiles, std::vector<int> *active) {
    std::vector<int> order(tubes.size());
    std::iota(order.begin(), order.end(), 0);
    auto rounds = [&](int t) { return (steps[t] + H - 1) / H; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rounds(a) > rounds(b); });
    tiles->clear();
    std::vector<int> tile_rounds;
    for (int t : order) {
        if (steps[t] <= 0) continue;
        for (int x0 = 0; x0 < tubes[t].nx; x0 += S) {
            tiles->push_back(BatchTile{t, x0, std::min(S, tubes[t].nx - x0), 0});
            tile_rounds.push_back(rounds(t));
        }
    }
    const int R = tile_rounds.empty() ? 0 : tile_rounds.front();
    active->assign(R, 0);
    for (int r = 0; r < R; ++r)
        active->at(r) = (int)std::count_if(tile_rounds.begin(), tile_rounds.end(), [&](int k) { return k > r; });
}

}  // namespace

struct lbm_batch_s {
    lbm_batch_options opt{};
    Model model{};
    BatchLayout lay{};
    int ntubes = 0, fp64 = 0;
    double rho_ref = 1.0;
    std::vector<lbm_tube> tubes;
    std::vector<int64_t> cell_off;
    char *ws = nullptr;
    void *buf0 = nullptr, *buf1 = nullptr;
    BatchTube *d_tubes = nullptr;
    BatchTile *d_tiles_run = nullptr, *d_tiles_adv = nullptr;
    int *d_steps_run = nullptr, *d_steps_adv = nullptr, *d_bad = nullptr;
    int *d_list = nullptr;  // active tiles of a device-driven schedule: count, then tile indices
    unsigned char *d_mask = nullptr;
    std::vector<int> active_run, active_adv;
    bool run_odd = false;  // some tube of the run schedule takes an odd number of rounds
    std::vector<int> adv_steps_host;
    std::vector<BatchTile> adv_tiles_host;
    hipStream_t stream = nullptr, cap = nullptr;
    hipGraphExec_t graph = nullptr;
    int64_t updates_run = 0;
};

namespace {

// the launches of one schedule: set the step counts (unless steps is null: the
// device set them, with the list of the active tiles, in batch_decide_dev), the
// rounds, and the flip of the tubes that ran an odd number of rounds (when any
// can).  With a device-decided schedule the rounds' first workgroups take
// exactly the listed tiles and the others return at once, after them.
hipError_t enqueue_schedule(lbm_batch_s *b, const BatchTile *tiles, const int *steps,
                            const std::vector<int> &active, bool odd_rounds, hipStream_t s) {
    const int W = b->lay.S + 2 * b->lay.H;
    hipError_t e = hipSuccess;
    if (steps) e = batch_set_steps(b->d_tubes, b->ntubes, steps, s);
    const int *list = steps ? nullptr : b->d_list;
    for (int r = 0; r < (int)active.size() && e == hipSuccess; ++r)
        e = batch_round(b->fp64, b->buf0, b->buf1, b->d_tubes, tiles, list, active[r], r, b->lay.H, W, b->lay.block,
                        b->model, b->rho_ref, s);
    if (e == hipSuccess && odd_rounds) e = batch_flip(b->d_tubes, b->ntubes, b->lay.H, s);
    return e;
}

// true when some tube of a host schedule runs an odd number of rounds
bool any_odd_rounds(const std::vector<int> &steps, int H) {
    for (int v : steps)
        if (((v + H - 1) / H) & 1) return true;
    return false;
}

bool uniform_nx(const lbm_batch_s *b) {
    for (const auto &t : b->tubes)
        if (t.nx != b->tubes[0].nx) return false;
    return true;
}

}  // namespace

namespace lbm {
// stream of a batch (the surrogate's hybrid advance runs on the same stream)
hipStream_t batch_stream(const lbm_batch_s *b) { return b->stream; }
// number of tubes and their common length (-1 when the lengths differ)
void batch_shape(const lbm_batch_s *b, int *ntubes, int *nx) {
    *ntubes = b->ntubes;
    *nx = b->tubes.empty() ? -1 : b->tubes[0].nx;
    for (const auto &t : b->tubes)
        if (t.nx != *nx) *nx = -1;
}

// Device-driven masking for the surrogate's hybrid advance.  The schedule of
// every tube at nsteps steps is uploaded once (synchronizing first, since the
// host staging vectors are reused); batch_decide_dev then writes, per jump, the
// tube mask (d_mask, read by batch_commit_dev), the step counts (0 or nsteps)
// and the list of the active tiles: tiles of a tube with 0 steps return at once
// and its buffer does not flip, so the host never waits on a decision.
hipError_t batch_device_schedule(lbm_batch_s *b, int nsteps) {
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return e;
    b->adv_steps_host.assign(b->ntubes, nsteps);
    schedule(b->tubes, b->adv_steps_host, b->lay.S, b->lay.H, &b->adv_tiles_host, &b->active_adv);
    if (!b->adv_tiles_host.empty())
        e = hipMemcpyAsync(b->d_tiles_adv, b->adv_tiles_host.data(), sizeof(BatchTile) * b->adv_tiles_host.size(),
                           hipMemcpyHostToDevice, b->stream);
    return e;
}
// Profiles of the tubes whose skip flag is clear (for a batch of tubes of equal
// length; the others keep theirs).
hipError_t batch_profiles_dev(lbm_batch_s *b, float *prof_dev, const unsigned char *skip) {
    return batch_profiles(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, prof_dev, b->rho_ref, b->stream, skip);
}
// Populations of the tubes with mask[t] set to f_eq of their profiles.
hipError_t batch_set_profiles_dev(lbm_batch_s *b, const unsigned char *mask, const float *prof_dev) {
    return batch_set_profiles(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, mask, prof_dev, b->model, b->rho_ref,
                              b->stream);
}
// After batch_decide_dev: accepted tubes keep pout as their state (pin = pout,
// lazy set); rejected tubes whose state was a profile get their populations
// from it before the rounds (lazy cleared).
hipError_t batch_commit_dev(lbm_batch_s *b, unsigned char *lazy, float *pin, const float *pout) {
    return batch_commit(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, b->d_mask, lazy, pin, pout, b->model,
                        b->rho_ref, b->stream);
}
// The decision of a device-driven schedule from per-tube indicators (accepted:
// finite and <= tol, no steps; rejected: nsteps of the schedule), the tube mask
// and the list of the rejected tubes' tiles, in one kernel; *count_dev = the
// number rejected.  Then batch_rounds_dev runs the rounds.
hipError_t batch_decide_dev(lbm_batch_s *b, const float *resid_dev, float tol, int *count_dev) {
    const int ntiles = b->active_adv.empty() ? 0 : b->active_adv[0];
    const int nsteps = b->adv_steps_host.empty() ? 0 : b->adv_steps_host[0];
    return batch_decide_list(resid_dev, b->ntubes, tol, nsteps, b->d_mask, b->d_tubes, b->d_tiles_adv, ntiles,
                             b->d_list, count_dev, b->stream);
}
hipError_t batch_rounds_dev(lbm_batch_s *b) {
    if (b->adv_tiles_host.empty()) return hipSuccess;
    return enqueue_schedule(b, b->d_tiles_adv, nullptr, b->active_adv, any_odd_rounds(b->adv_steps_host, b->lay.H),
                            b->stream);
}
}  // namespace lbm

extern "C" {

lbm_status lbm_batch_workspace_bytes(const lbm_tube *tubes, int ntubes, const lbm_batch_options *opt,
                                     size_t *bytes) {
    if (!bytes) return bfail(LBM_ERR_ARG, "null argument");
    Model m;
    BatchLayout lay;
    lbm_status s = check(tubes, ntubes, opt, &m, &lay);
    if (s != LBM_OK) return s;
    *bytes = lay.total;
    return LBM_OK;
}

lbm_status lbm_batch_init(const lbm_tube *tubes, int ntubes, const lbm_batch_options *opt, void *workspace,
                          size_t bytes, void *stream, lbm_batch *out) {
    if (!workspace || !out) return bfail(LBM_ERR_ARG, "null argument");
    *out = nullptr;
    Model m;
    BatchLayout lay;
    lbm_status s = check(tubes, ntubes, opt, &m, &lay);
    if (s != LBM_OK) return s;
    if (bytes < lay.total) return bfail(LBM_ERR_ARG, "workspace smaller than lbm_batch_workspace_bytes()");
    if ((uintptr_t)workspace % kAlign) return bfail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
    lbm_batch_s *b = new (std::nothrow) lbm_batch_s;
    if (!b) return bfail(LBM_ERR_ARG, "out of host memory");
    b->opt = *opt;
    b->model = m;
    b->lay = lay;
    b->ntubes = ntubes;
    b->fp64 = opt->precision == LBM_FP64;
    b->rho_ref = opt->rho_ref > 0 ? opt->rho_ref : 1.0;
    b->tubes.assign(tubes, tubes + ntubes);
    b->stream = (hipStream_t)stream;
    b->ws = (char *)workspace;
    b->buf0 = b->ws;
    b->buf1 = b->ws + lay.buf;
    b->d_tubes = (BatchTube *)(b->ws + lay.off_tubes);
    b->d_tiles_run = (BatchTile *)(b->ws + lay.off_tiles_run);
    b->d_steps_run = (int *)(b->ws + lay.off_steps_run);
    b->d_tiles_adv = (BatchTile *)(b->ws + lay.off_tiles_adv);
    b->d_steps_adv = (int *)(b->ws + lay.off_steps_adv);
    b->d_mask = (unsigned char *)(b->ws + lay.off_mask);
    b->d_bad = (int *)(b->ws + lay.off_bad);
    b->d_list = (int *)(b->ws + lay.off_list);

    std::vector<BatchTube> ht(ntubes);
    std::vector<int> steps(ntubes);
    int64_t cell = 0;
    b->cell_off.resize(ntubes + 1);
    for (int t = 0; t < ntubes; ++t) {
        ht[t] = BatchTube{cell * Q, tubes[t].nx, 0, 0, 0, 1.0 / tubes[t].tau, tubes[t].n_left, tubes[t].n_right};
        b->cell_off[t] = cell;
        cell += (int64_t)NY * tubes[t].nx;
        steps[t] = (int)tubes[t].steps;
        b->updates_run += (int64_t)NY * tubes[t].nx * tubes[t].steps;
    }
    b->cell_off[ntubes] = cell;
    std::vector<BatchTile> tiles;
    schedule(b->tubes, steps, lay.S, lay.H, &tiles, &b->active_run);
    b->run_odd = any_odd_rounds(steps, lay.H);
    hipError_t e = hipMemcpyAsync(b->d_tubes, ht.data(), sizeof(BatchTube) * ntubes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpyAsync(b->d_tiles_run, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_steps_run, steps.data(), sizeof(int) * ntubes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // the host vectors go out of scope
    if (e == hipSuccess) e = batch_init(b->fp64, b->buf0, b->buf1, b->d_tubes, ntubes, m, b->rho_ref, b->stream);
    if (e != hipSuccess) {
        delete b;
        return bhip(e, "batch init");
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch b) {
    if (!b) return bfail(LBM_ERR_ARG, "null batch");
    hipError_t e;
    if (!b->opt.use_graph) {
        e = enqueue_schedule(b, b->d_tiles_run, b->d_steps_run, b->active_run, b->run_odd, b->stream);
        return e == hipSuccess ? LBM_OK : bhip(e, "batch run");
    }
    if (!b->graph) {
        if (!b->cap) {
            e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
            if (e != hipSuccess) return bhip(e, "hipStreamCreateWithFlags");
        }
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return bhip(e, "hipStreamBeginCapture");
        hipError_t le = enqueue_schedule(b, b->d_tiles_run, b->d_steps_run, b->active_run, b->run_odd, b->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bhip(le, "launch during capture");
        }
        if (e != hipSuccess) return bhip(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return bhip(e, "hipGraphInstantiate");
    }
    e = hipGraphLaunch(b->graph, b->stream);
    return e == hipSuccess ? LBM_OK : bhip(e, "hipGraphLaunch");
}

lbm_status lbm_batch_advance(lbm_batch b, int64_t nsteps, const unsigned char *active_host) {
    if (!b) return bfail(LBM_ERR_ARG, "null batch");
    if (nsteps < 0 || nsteps > 0x3fffffff) return bfail(LBM_ERR_ARG, "nsteps out of range");
    if (nsteps == 0) return LBM_OK;
    // the host staging vectors are reused: wait for the previous upload to be consumed
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(e, "hipStreamSynchronize");
    b->adv_steps_host.assign(b->ntubes, 0);
    for (int t = 0; t < b->ntubes; ++t)
        if (!active_host || active_host[t]) b->adv_steps_host[t] = (int)nsteps;
    schedule(b->tubes, b->adv_steps_host, b->lay.S, b->lay.H, &b->adv_tiles_host, &b->active_adv);
    if (b->adv_tiles_host.empty()) return LBM_OK;
    e = hipMemcpyAsync(b->d_tiles_adv, b->adv_tiles_host.data(), sizeof(BatchTile) * b->adv_tiles_host.size(),
                       hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_steps_adv, b->adv_steps_host.data(), sizeof(int) * b->ntubes, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess)
        e = enqueue_schedule(b, b->d_tiles_adv, b->d_steps_adv, b->active_adv,
                             any_odd_rounds(b->adv_steps_host, b->lay.H), b->stream);
    return e == hipSuccess ? LBM_OK : bhip(e, "batch advance");
}

lbm_status lbm_batch_set_equilibrium(lbm_batch b, const double *n_dev, const double *u_dev,
                                     const unsigned char *mask_host) {
    if (!b || !n_dev || !u_dev) return bfail(LBM_ERR_ARG, "null argument");
    hipError_t e = hipStreamSynchronize(b->stream);
    std::vector<unsigned char> mask(b->ntubes, 1);
    if (mask_host) mask.assign(mask_host, mask_host + b->ntubes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_mask, mask.data(), b->ntubes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = batch_set_eq(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, b->d_mask, n_dev, u_dev, b->lay.cells,
                         b->model, b->rho_ref, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // mask leaves scope
    return e == hipSuccess ? LBM_OK : bhip(e, "batch set equilibrium");
}

lbm_status lbm_batch_moments(lbm_batch b, double *n_dev, double *u_dev) {
    if (!b || !n_dev || !u_dev) return bfail(LBM_ERR_ARG, "null argument");
    hipError_t e = batch_moments(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, n_dev, u_dev, b->d_bad,
                                 b->lay.cells, b->rho_ref, b->stream);
    return e == hipSuccess ? LBM_OK : bhip(e, "batch moments");
}

lbm_status lbm_batch_health(lbm_batch b, int *bad_cells_host) {
    if (!b || !bad_cells_host) return bfail(LBM_ERR_ARG, "null argument");
    hipError_t e = batch_moments(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, nullptr, nullptr, b->d_bad,
                                 b->lay.cells, b->rho_ref, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bad_cells_host, b->d_bad, sizeof(int) * b->ntubes, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? LBM_OK : bhip(e, "batch health");
}

lbm_status lbm_batch_profiles(lbm_batch b, float *prof_dev) {
    if (!b || !prof_dev) return bfail(LBM_ERR_ARG, "null argument");
    if (!uniform_nx(b)) return bfail(LBM_ERR_UNSUPPORTED, "profiles need tubes of equal length");
    hipError_t e = batch_profiles(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, prof_dev, b->rho_ref, b->stream);
    return e == hipSuccess ? LBM_OK : bhip(e, "batch profiles");
}

lbm_status lbm_batch_set_profiles(lbm_batch b, const float *prof_dev, const unsigned char *mask_host) {
    if (!b || !prof_dev) return bfail(LBM_ERR_ARG, "null argument");
    if (!uniform_nx(b)) return bfail(LBM_ERR_UNSUPPORTED, "profiles need tubes of equal length");
    hipError_t e = hipStreamSynchronize(b->stream);
    std::vector<unsigned char> mask(b->ntubes, 1);
    if (mask_host) mask.assign(mask_host, mask_host + b->ntubes);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_mask, mask.data(), b->ntubes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = batch_set_profiles(b->fp64, b->buf0, b->buf1, b->d_tubes, b->ntubes, b->d_mask, prof_dev, b->model,
                               b->rho_ref, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // mask leaves scope
    return e == hipSuccess ? LBM_OK : bhip(e, "batch set profiles");
}

lbm_status lbm_batch_layout(lbm_batch b, int64_t *cell_offsets_host) {
    if (!b || !cell_offsets_host) return bfail(LBM_ERR_ARG, "null argument");
    std::copy(b->cell_off.begin(), b->cell_off.end(), cell_offsets_host);
    return LBM_OK;
}

lbm_status lbm_batch_info(lbm_batch b, int64_t *total_cells, int64_t *updates_per_run, int *rounds, int *tile_cols,
                          int *halo) {
    if (!b || !total_cells || !updates_per_run || !rounds || !tile_cols || !halo)
        return bfail(LBM_ERR_ARG, "null argument");
    *total_cells = b->lay.cells;
    *updates_per_run = b->updates_run;
    *rounds = (int)b->active_run.size();
    *tile_cols = b->lay.S;
    *halo = b->lay.H;
    return LBM_OK;
}

lbm_status lbm_batch_free(lbm_batch b) {
    if (!b) return LBM_OK;
    lbm_status st = LBM_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) st = bhip(e, "hipStreamSynchronize");
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return st;
}

}  // extern "C"
