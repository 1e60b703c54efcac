// Host runtime and C ABI of the parabolic sub-step (see include/tlim.h).
//
// The runtime owns no device memory: the caller binds one workspace and the
// context carves its fields and scratch out of it.  It computes the LIM
// schedule on the host from the Gershgorin bound read back once per Picard
// pass (the count of sweeps 2P-1 decides how many launches follow), and
// enqueues everything else on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tlim.h"
#include "tlim_internal.h"
#include "tlim_sweep.h"

using tlim::DevGrid;
using tlim::DevPhases;
using tlim::PassResult;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
constexpr int kMaxEvents = 2 * (TLIM_MAX_PASSES + 4);
constexpr int kStepPmax = 256;  // largest P of the whole-step kernel's parameter table

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct tlim_ctx {
    int64_t n[3];
    double h[3];
    int32_t bc[3];
    int64_t N;
    int precision;
    hipStream_t stream;
    int device;
    tlim_phase phase[2];
    bool phase_set[2];
    // workspace
    char* ws;
    size_t ws_bytes;
    double* field[TLIM_NFIELDS];
    bool fset[TLIM_NFIELDS];
    double *Tn, *Tnew, *a2n, *Lam, *rC, *rhs, *vb[2];
    double* Lam_alt;  // the next pass's conductivities, built by the pass before
    const double* g_heat;  // right-hand side g of the heat passes: rhs, or Tn when there is no source
    float *Lam32, *rC32, *q32, *wb[2];
    float *Lam32_alt, *q32_alt;  // the next pass's float coefficients, built by the pass before
    float* wzero;                // all zero: the correction form's start w0 = T^n - g without sources
    // The last launch of an FP64 step has relaxed the next step's state and
    // built its first coefficients (valid until the state or the phases
    // change); spare_clean: the row of that bound is zero.
    // row0_moved: the step-end fold moved that bound into the first pass's
    // row (zero it before any other use).
    bool next_ready, spare_clean, row0_moved;
    double next_eps;
    double* chat_tab;            // whole-step kernel: b/lambda per P (order chat_order, -1: not built)
    int chat_order;
    unsigned* bar;               // whole-step kernel: barrier counter
    unsigned* collect_done;      // folds that publish a sequence number: workgroups done
    unsigned long long res_seq;  // last sequence number given to such a fold
    bool w0_zero;                // the coefficients of the current pass came without sources
    double* acc;           // reduction rows: kTargets x kSlots
    PassResult* res_dev;   // folded results (one double per target)
    PassResult* res_host;  // pinned copy (the current block of res_blk)
    PassResult* res_host_dev;  // device address of res_host (NULL: copy from res_dev)
    PassResult* res_blk[2];    // two pinned result blocks: a pipelined step keeps its own
    PassResult* res_blk_dev[2];
    int res_cur;
    // T^n of consecutive steps rotate through three arrays and the relaxed
    // alpha2 through the alpha2 field, a2n and a2x: a step's T^n and alpha2
    // outlive the enqueue of the next step and of the one after it (whose
    // start a step's last launch may build ahead of time).
    double* Tn_buf[3];
    double* a2x;
    double* a2pool[3];  // the three alpha2 arrays
    double *next_tn, *next_a2;  // where the next step's start was built
    // A predicted step enqueued without waiting for its readback (pipelined
    // mode); it is verified by the next call.
    bool pending;
    struct Pending {
        tlim_step_opts o;
        int P_used[TLIM_MAX_PASSES];
        int blk;                // its result block
        double* Tn;             // its relaxed T
        double* alpha2;         // its relaxed alpha2 (the alpha2 field during its passes)
        double* alpha2_other;   // the other alpha2 array
        bool whole;             // run by the whole-step kernel (P decided on the device)
        unsigned long long seq; // nonzero: its fold publishes seq in its result block (no event)
    } pend;
    hipEvent_t ev_pend[2];
    // Leading rows of the Picard-pass targets known to be zero, and the count
    // to restore when the step's final readback consumes its rows.
    int clean_rows, clean_keep;
    hipEvent_t ev[kMaxEvents];
    hipEvent_t ev_sync;  // readback completion (polled)
    // Schedule history for P prediction: P of each Picard pass of the last
    // completed step (hist_passes = 0: none).
    int hist_passes;
    int hist_P[TLIM_MAX_PASSES];
    // lambda_G per pass of the last verified step (hist_nlam = 1: present)
    double hist_lam[TLIM_MAX_PASSES];
    int hist_nlam;
    // Consecutive verified steps whose passes all ran the P of the step
    // before's last pass (a schedule settled enough to pipeline).
    int hist_steady;
    // After a step T_2 = T_1 everywhere: the T2 field then reads through T1.
    bool t2_alias;
    int64_t predict_misses;
    int64_t pipelined_steps, pipeline_redos;
    // Polls a grid-barrier wait of the whole-step kernel may take before it
    // counts a time-out (about a second by default).
    unsigned step2d_spin_limit;
    std::string err;
};

namespace {

tlim_status fail(tlim_ctx* c, tlim_status s, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIP_TRY(c, expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail((c), TLIM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// A grid-barrier wait of the whole-step kernel timed out.  Workgroups that
// stopped waiting may have written a pass's T^(it+1) into the T1 field while
// another workgroup had not yet read it for its relaxation, so neither the
// step's result nor its relaxed start can be trusted.  Wait for everything
// enqueued (a pipelined step after it included), drop it, and mark the
// fields the heat step writes (alpha2, T1, T2) as not set: the next call
// that needs them returns TLIM_E_STATE until the caller sets them again.
tlim_status lose_heat_state(tlim_ctx* c) {
    (void)hipStreamSynchronize(c->stream);
    c->pending = false;
    c->next_ready = false;
    c->t2_alias = false;
    c->fset[TLIM_ALPHA2] = c->fset[TLIM_T1] = c->fset[TLIM_T2] = false;
    return fail(c, TLIM_E_HIP, "whole-step kernel: barrier time-out; alpha2, T1 and T2 are lost and must be set again");
}

// Layout of the workspace: byte offsets of every array (all 256-aligned).
struct Layout {
    size_t field[TLIM_NFIELDS];
    size_t Tn, Tn2, Tn3, Tnew, a2n, a2x, Lam, Lam2, rC, rhs, vb[2], acc, res;
    size_t Lam32, rC32, q32, wb[2], Lam32b, q32b, wzero;
    size_t chat, bar, cnt;
    size_t total;
};

Layout layout_of(const int64_t n[3], int precision) {
    const int64_t N = n[0] * n[1] * n[2];
    Layout L{};
    size_t off = 0;
    size_t d = align_up(sizeof(double) * (size_t)N), f = align_up(sizeof(float) * (size_t)N);
    for (int i = 0; i < TLIM_NFIELDS; ++i) {
        L.field[i] = off;
        off += d;
    }
    size_t* dd[] = {&L.Tn, &L.Tn2, &L.Tn3, &L.Tnew, &L.a2n, &L.a2x, &L.Lam, &L.Lam2, &L.rC, &L.rhs, &L.vb[0],
                    &L.vb[1]};
    for (size_t* p : dd) {
        *p = off;
        off += d;
    }
    L.acc = off;
    off += align_up(sizeof(double) * (size_t)tlim::kTargets * tlim::kSlots);
    L.res = off;
    off += align_up(sizeof(PassResult));
    L.chat = off;
    off += align_up(sizeof(double) * (size_t)kStepPmax * kStepPmax);
    L.bar = off;
    off += align_up(sizeof(unsigned) * tlim::kStepMaxTiles);
    L.cnt = off;
    off += align_up(sizeof(double));
    if (precision == TLIM_FP32) {
        size_t* ff[] = {&L.Lam32, &L.rC32, &L.q32, &L.wb[0], &L.wb[1], &L.Lam32b, &L.q32b, &L.wzero};
        for (size_t* p : ff) {
            *p = off;
            off += f;
        }
    }
    L.total = off;
    return L;
}

DevGrid dev_grid(const tlim_ctx* c, const double scale[3]) {
    DevGrid g{};
    g.nx = (int)c->n[0];
    g.ny = (int)c->n[1];
    g.nz = (int)c->n[2];
    for (int d = 0; d < 3; ++d) {
        g.per[d] = c->bc[d] == TLIM_PERIODIC;
        g.w[d] = scale[d] / (c->h[d] * c->h[d]);
    }
    g.N = c->N;
    return g;
}

const double kUnit[3] = {1.0, 1.0, 1.0};

DevPhases dev_phases(const tlim_ctx* c) { return tlim::pack_phases(c->phase); }

// ---------------------------------------------------------------- schedule

// Number of Chebyshev parameters of one LIM pass (Sec. 3.2).
int lim_P(double tau, double lambda_max) { return (int)std::ceil(kPi / 4.0 * std::sqrt(tau * lambda_max + 1.0)); }

// Parameters b_1..b_{2P-1} (Sec. 3.2): a_j = lambda (beta_1 - beta_j)/(1 + beta_1)
// with beta_j = cos((2j-1) pi/(2P)) the roots of T_P, beta_1 the largest.  The
// inner 2P-2 stages use every a_j (j >= 2) twice; order selects their sequence,
// the last stage is always a_1 = 0.
std::vector<double> lim_params(int P, double lambda_max, int order) {
    std::vector<double> a(P + 1, 0.0);
    const double beta1 = std::cos(kPi / (2.0 * P));
    for (int j = 2; j <= P; ++j) a[j] = lambda_max / (1.0 + beta1) * (beta1 - std::cos((2.0 * j - 1.0) * kPi / (2.0 * P)));
    std::vector<double> b;
    b.reserve(2 * P - 1);
    if (order == TLIM_ORDER_PAPER) {
        for (int j = P; j >= 2; --j) b.push_back(a[j]);
        for (int j = P; j >= 2; --j) b.push_back(a[j]);
    } else if (order == TLIM_ORDER_ASCENDING) {
        for (int j = 2; j <= P; ++j) {
            b.push_back(a[j]);
            b.push_back(a[j]);
        }
    } else {
        // largest, smallest, second largest, second smallest, ... (twice): keeps
        // every partial product of stage factors bounded, so round-off stays at
        // the tau*lambda*eps floor of the final explicit stage
        std::vector<double> once;
        int lo = 2, hi = P;
        bool take_hi = true;
        while (lo <= hi) {
            once.push_back(take_hi ? a[hi--] : a[lo++]);
            take_hi = !take_hi;
        }
        b.insert(b.end(), once.begin(), once.end());
        b.insert(b.end(), once.begin(), once.end());
    }
    b.push_back(0.0);
    return b;
}

// Chebyshev-Richardson cycle of s stages: 1 + tau b_j at the Chebyshev nodes
// of [1, 1 + tau lambda], increasing.
std::vector<double> cycle_params(int s, double lambda_max) {
    std::vector<double> b(s);
    for (int k = 0; k < s; ++k) b[k] = 0.5 * lambda_max * (1.0 + std::cos((2.0 * (s - k) - 1.0) * kPi / (2.0 * s)));
    return b;
}

// b/lambda of every P <= kStepPmax for the stage order, at offset (P-1)^2.
// Built when a context binds its workspace (default order) or when a step
// asks for another order; the upload waits for the stream.
tlim_status step2d_table(tlim_ctx* c, int order) {
    if (c->chat_order == order) return TLIM_OK;
    std::vector<double> t((size_t)kStepPmax * kStepPmax, 0.0);
    for (int P = 1; P <= kStepPmax; ++P) {
        const std::vector<double> ch = lim_params(P, 1.0, order);
        std::copy(ch.begin(), ch.end(), t.begin() + (size_t)(P - 1) * (P - 1));
    }
    HIP_TRY(c, hipMemcpyAsync(c->chat_tab, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->chat_order = order;
    return TLIM_OK;
}

// ------------------------------------------------------------------ checks

tlim_status check_ready(tlim_ctx* c, bool need_T = true) {
    if (!c->ws) return fail(c, TLIM_E_STATE, "no workspace bound");
    if (!c->phase_set[0] || !c->phase_set[1]) return fail(c, TLIM_E_STATE, "both phases must be set");
    const int need[] = {TLIM_ALPHA2, TLIM_M1, TLIM_M2, TLIM_T1, TLIM_T2};
    for (int f : need)
        if (need_T && !c->fset[f]) return fail(c, TLIM_E_STATE, "field %d not set", f);
    return TLIM_OK;
}

tlim_status check_opts(tlim_ctx* c, const tlim_step_opts* o) {
    if (!o) return fail(c, TLIM_E_ARG, "opts is NULL");
    if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(c, TLIM_E_ARG, "dt must be finite and > 0");
    if (o->passes < 1 || o->passes > TLIM_MAX_PASSES) return fail(c, TLIM_E_ARG, "passes out of range");
    if (o->picard_tol < 0.0) return fail(c, TLIM_E_ARG, "picard_tol < 0");
    if (o->order < 0 || o->order > 2) return fail(c, TLIM_E_ARG, "unknown order");
    if (o->face_mean < 0 || o->face_mean > 1) return fail(c, TLIM_E_ARG, "unknown face_mean");
    if (o->alpha_eps < 0.0 || o->alpha_eps >= 0.5) return fail(c, TLIM_E_ARG, "alpha_eps out of [0, 0.5)");
    if (o->cycle_mode && (o->max_cycles < 1 || !(o->cycle_tol >= 0.0)))
        return fail(c, TLIM_E_ARG, "cycle mode needs max_cycles >= 1 and cycle_tol >= 0");
    if (o->cycle_mode && c->precision != TLIM_FP64) return fail(c, TLIM_E_ARG, "cycle mode runs in FP64 contexts");
    if (o->do_viscous) {
        for (int d = 0; d < 3; ++d)
            if (c->n[d] > 1 && !c->fset[TLIM_U + d]) return fail(c, TLIM_E_STATE, "velocity component %d not set", d);
    }
    if (o->frozen_lambda)
        for (int i = 0; i < o->passes; ++i)
            if (!(o->frozen_lambda[i] >= 0.0) || !std::isfinite(o->frozen_lambda[i]))
                return fail(c, TLIM_E_ARG, "frozen_lambda[%d] invalid", i);
    return TLIM_OK;
}

// ---------------------------------------------------------- one LIM pass

// Kernel time of the sweep launches (time_sweeps): a pair of events around
// each run of back-to-back sweep launches; when the pairs run out the
// elapsed times so far are folded (which waits for them) and the events are
// reused.
struct Timer {
    tlim_ctx* c;
    bool on;
    bool skip = false;  // the next run follows a readback: not timed
    int used = 0;
    double folded_ms = 0.0;
    void start() {
        if (!on || skip) return;
        if (used + 1 >= kMaxEvents) fold();
        (void)hipEventRecord(c->ev[used], c->stream);
    }
    void stop() {
        if (!on || skip) return;
        (void)hipEventRecord(c->ev[used + 1], c->stream);
        used += 2;
    }
    void fold() {
        if (used > 0) (void)hipEventSynchronize(c->ev[used - 1]);
        for (int i = 0; i + 1 < used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]) == hipSuccess) folded_ms += ms;
        }
        used = 0;
    }
    void reset() {
        used = 0;
        folded_ms = 0.0;
    }
    double elapsed_ms() {
        fold();
        return folded_ms;
    }
};

struct SweepCount {
    int64_t sweeps = 0, launches = 0;
    int64_t timed_sweeps = 0, timed_launches = 0;  // inside the timer's event pairs
};

// Reduction rows are zeroed before the kernels that accumulate into them
// (stream order); collect folds them for the host.
double* row(tlim_ctx* c, int t) { return c->acc + (size_t)t * tlim::kSlots; }
void zero_rows(tlim_ctx* c, int t0, int t1) { tlim::launch_zero_rows(c->stream, c->acc, t0, t1); }
double result(const tlim_ctx* c, int t) { return c->res_host->v[t]; }

// The reduction rows of pass it.  With dmax = false the Picard change is not
// formed (its row stays zero and the kernels do not read T^(it)): a step
// without a report and without a Picard tolerance never reads it.
tlim::PassSlots pass_slots(tlim_ctx* c, int it, bool dmax = true) {
    return tlim::PassSlots{dmax ? row(c, tlim::tgt_dmax(it)) : nullptr, row(c, tlim::tgt_tmax(it)),
                           row(c, tlim::tgt_bad(it))};
}

double* T2_ptr(tlim_ctx* c) { return c->t2_alias ? c->field[TLIM_T1] : c->field[TLIM_T2]; }

// Stage parameters of one pass: given b (lam_dev == NULL) or, with the
// bound on the device, the normalised parameters b/lambda of the same P.
struct PassSchedule {
    const double* lam_dev = nullptr;
    std::vector<double> tb;    // tau * b_m (host bound)
    std::vector<double> chat;  // b_m / lambda (device bound)
    int nst = 0;
    tlim::Stages at(int m) const {
        tlim::Stages st;
        st.lam = lam_dev;
        st.tb = lam_dev ? nullptr : tb.data() + m;
        st.chat = lam_dev ? chat.data() + m : nullptr;
        return st;
    }
};

PassSchedule host_schedule(double tau, double lam, int order) {
    PassSchedule ps;
    int P = lim_P(tau, lam);
    std::vector<double> b = lim_params(P, lam, order);
    ps.nst = (int)b.size();
    ps.tb.resize(b.size());
    for (size_t m = 0; m < b.size(); ++m) ps.tb[m] = tau * b[m];
    return ps;
}

PassSchedule device_schedule(int P, int order, const double* lam_dev) {
    PassSchedule ps;
    ps.chat = lim_params(P, 1.0, order);
    ps.nst = (int)ps.chat.size();
    ps.lam_dev = lam_dev;
    return ps;
}

// out = LIM pass (eqs. LIM, LIM_last) from v0 with right-hand side rhs and the
// coefficients in c->Lam/c->rC (and their float copies in FP32 contexts).
// With Tit != NULL the kernel that writes `out` also accumulates the pass
// reductions into ps.
// In FP32 contexts q and w0 come from the heat coefficient kernel
// (have_q = true) or are built here.
// The predicted iterate v^(2P-2) of a pass run with its final stage on its
// own (uh64, or g64 + w32 in FP32 contexts).
struct Vhat {
    const double* v64 = nullptr;
    const double* g64 = nullptr;
    const float* w32 = nullptr;
};

// nc (FP64, nullable): the launch that reaches the final stage also builds
// the next pass's coefficients when it can; *nc_done tells whether it did.
void run_lim_pass(tlim_ctx* c, const DevGrid& g, int face, double tau, const PassSchedule& ps, const double* v0,
                  const double* rhs, double* out, const double* Tit, tlim::PassSlots slots, Timer& tm,
                  SweepCount& sc, bool have_q = false, Vhat* vh = nullptr, const tlim::NextCoef* nc = nullptr,
                  bool* nc_done = nullptr) {
    if (nc_done) *nc_done = false;
    const int nst = ps.nst;
    hipStream_t s = c->stream;
    // a pass that starts from its own source (v0 = rhs: the viscous part)
    // has w0 = v0 - rhs = 0: it starts from the zero array
    const bool zero_start = c->precision == TLIM_FP32 && v0 == rhs && c->wzero != nullptr;
    if (c->precision == TLIM_FP32 && !have_q)
        tlim::launch_q32(s, g, face, rhs, v0, c->Lam32, c->rC32, tau, c->q32, zero_start ? nullptr : c->wb[0]);
    // one event pair around the pass's back-to-back sweep launches
    const int64_t launches0 = sc.launches;
    tm.start();
    if (c->precision == TLIM_FP32) {
        // 2P-2 float stages on the correction, the final one in double; the
        // launch that reaches it writes `out`
        // w0 = 0 without sources: start from the zero array (no write needed)
        const float* cur = (have_q && c->w0_zero) || zero_start ? c->wzero : c->wb[0];
        int m = 0;
        const int upto = vh ? nst - 1 : nst;  // with vh the final stage runs on its own
        // (stage 1 must be a float stage: the final stage is the last of
        // upto unless vh takes it)
        if (cur == c->wzero && tlim::use_z3d(g) && upto >= (vh ? 2 : 3)) {
            // one stage per launch on 3D grids: the first stage from w = 0 is
            // c_0 q exactly, so it rides along with the second
            auto sp = [&](int k) {
                return ps.lam_dev ? tlim::StageParam{ps.lam_dev, 0.0, ps.chat[k]}
                                  : tlim::StageParam{nullptr, ps.tb[k], 0.0};
            };
            tlim::launch_z3d_two_from_zero32(s, g, face, c->q32, c->Lam32, c->rC32, c->wb[0], sp(0), sp(1), tau);
            cur = c->wb[0];
            m = 2;
            sc.launches++;
        }
        while (m < upto) {
            int k = tlim::sweeps_per_launch(g, upto - m);
            bool last = !vh && m + k == nst;
            float* nxt = cur == c->wb[0] ? c->wb[1] : c->wb[0];
            int done = tlim::launch_sweeps32(s, g, face, cur, c->q32, c->Lam32, c->rC32, nxt, ps.at(m), k, last, tau,
                                             rhs, c->rC, out, Tit, slots, last ? nc : nullptr,
                                             last ? nc_done : nullptr, cur == c->wzero);
            cur = nxt;
            m += done;
            sc.launches++;
        }
        if (vh) {
            tlim::launch_final32(s, g, face, cur, rhs, c->Lam32, c->rC, out, tau, Tit, slots);
            sc.launches++;
            vh->g64 = rhs;
            vh->w32 = cur;
        }
    } else {
        // all 2P-1 stages, the last (b = 0) in flux form; the launch that
        // reaches it writes `out`
        const double* cur = v0;
        int m = 0;
        int pp = 0;
        const int upto = vh ? nst - 1 : nst;
        while (m < upto) {
            int k = tlim::sweeps_per_launch(g, upto - m);
            bool last = !vh && m + k == nst;
            double* nxt = last ? out : c->vb[pp];
            int done = tlim::launch_sweeps64(s, g, face, cur, rhs, c->Lam, c->rC, nxt, ps.at(m), k, last, tau, Tit,
                                             slots, last ? nc : nullptr, last ? nc_done : nullptr);
            cur = nxt;
            pp ^= 1;
            m += done;
            sc.launches++;
        }
        if (vh) {
            tlim::launch_final64(s, g, face, cur, rhs, c->Lam, c->rC, out, tau, Tit, slots);
            sc.launches++;
            vh->v64 = cur;
        }
    }
    tm.stop();
    sc.sweeps += nst;
    if (tm.on && !tm.skip) {
        sc.timed_sweeps += nst;
        sc.timed_launches += sc.launches - launches0;
    }
    tm.skip = false;
}

// Wait until the fold that carries sequence number seq has written its
// results into the pinned block res: its number arrives after its values.
// Past ~2 ms (or after a fault that stopped the stream) the stream is
// drained instead.  The readbacks sit on the critical path between steps,
// and an event there costs about 5 us of idle GPU.
hipError_t wait_fold(tlim_ctx* c, PassResult* res, unsigned long long seq, bool* seen) {
    const auto t0c = std::chrono::steady_clock::now();
    hipError_t r = hipSuccess;
    while (!(*seen = __atomic_load_n(&res->seq, __ATOMIC_ACQUIRE) == seq)) {
        if (std::chrono::steady_clock::now() - t0c > std::chrono::microseconds(2000)) {
            r = hipStreamSynchronize(c->stream);
            *seen = __atomic_load_n(&res->seq, __ATOMIC_ACQUIRE) == seq;
            break;
        }
    }
    return *seen ? hipSuccess : r;
}

// Fold the rows [t0, t1) and bring the results to the host (synchronises).
// With consume the rows are also cleared on the device.
tlim_status read_result(tlim_ctx* c, int t0, int t1, bool consume = false, int move_from = -1) {
    if (c->res_host_dev && t1 > t0) {
        // the fold writes straight into the pinned result block
        const unsigned long long seq = ++c->res_seq;
        tlim::launch_collect(c->stream, c->acc, c->res_host_dev, t0, t1, consume ? 1 : 0, move_from, seq,
                             c->collect_done);
        bool seen = false;
        const hipError_t e = wait_fold(c, c->res_host, seq, &seen);
        if (e != hipSuccess) return fail(c, TLIM_E_HIP, "readback: %s", hipGetErrorString(e));
        if (!seen) return fail(c, TLIM_E_HIP, "readback: the stream drained without the results");
        return TLIM_OK;
    }
    if (c->res_host_dev) {
        tlim::launch_collect(c->stream, c->acc, c->res_host_dev, t0, t1, consume ? 1 : 0, move_from);
    } else {
        tlim::launch_collect(c->stream, c->acc, c->res_dev, t0, t1, consume ? 1 : 0, move_from);
        HIP_TRY(c, hipMemcpyAsync(c->res_host, c->res_dev, sizeof(PassResult), hipMemcpyDeviceToHost, c->stream));
    }
    // The readbacks sit on the critical path between steps: poll the
    // completion for up to ~2 ms before falling back to a blocking wait.
    HIP_TRY(c, hipEventRecord(c->ev_sync, c->stream));
    hipError_t e = hipErrorNotReady;
    const auto t0c = std::chrono::steady_clock::now();
    while ((e = hipEventQuery(c->ev_sync)) == hipErrorNotReady) {
        if (std::chrono::steady_clock::now() - t0c > std::chrono::microseconds(2000)) {
            e = hipEventSynchronize(c->ev_sync);
            break;
        }
    }
    if (e != hipSuccess) return fail(c, TLIM_E_HIP, "readback: %s", hipGetErrorString(e));
    return TLIM_OK;
}

// Zero the rows of the Picard-pass targets a step uses, unless the previous
// step's final readback left them zero.
void begin_pass_rows(tlim_ctx* c, int passes) {
    if (c->row0_moved) {
        // a next-step bound that is not adopted: the rows are not clean
        c->row0_moved = false;
        c->clean_rows = 0;
    }
    const int need = tlim::tgt_lam(passes);
    if (c->clean_rows < need) zero_rows(c, tlim::tgt_lam(0), need);
    c->clean_keep = std::max(c->clean_rows, need);
    c->clean_rows = 0;  // until the step's rows are consumed
}

double cell_volume(const tlim_ctx* c) { return c->h[0] * c->h[1] * c->h[2]; }

// Viscous sub-step: rho du_c/dt = sum_d d_d(mu_cd d_d u_c), mu_cd = 4/3 mu on
// axis c (Sec. 3.2, eq. viscous1D extended per axis), one LIM pass per component.
tlim_status viscous(tlim_ctx* c, const tlim_step_opts* o, tlim_step_report* rep, Timer& tm, SweepCount& sc) {
    DevPhases ph = dev_phases(c);
    DevGrid g0 = dev_grid(c, kUnit);
    tlim::launch_visc_coeffs(c->stream, g0, ph, c->field[TLIM_ALPHA2], c->field[TLIM_M1], c->field[TLIM_M2], c->Lam,
                             c->rC, c->Lam32, c->rC32);
    const bool heat = o->visc_heating != 0;
    double* E = c->fset[TLIM_E] ? c->field[TLIM_E] : nullptr;
    if (heat) c->next_ready = false;  // T changes before the relaxation
    if (heat && c->t2_alias) {
        // the phases are heated differently: T2 gets its own array again
        tlim::launch_copy(c->stream, c->field[TLIM_T2], c->field[TLIM_T1], c->N);
        c->t2_alias = false;
    }
    // the components' bounds depend on (Lambda, 1/C) only, which the passes
    // do not change: all of them from one kernel and one readback
    double lam_c[3] = {0.0, 0.0, 0.0};
    if (!o->frozen_visc) {
        double wc[3][3];
        int mask = 0;
        for (int comp = 0; comp < 3; ++comp) {
            double scale[3] = {1.0, 1.0, 1.0};
            scale[comp] = 4.0 / 3.0;
            const DevGrid gc = dev_grid(c, scale);
            for (int d = 0; d < 3; ++d) wc[comp][d] = gc.w[d];
            if (c->n[comp] > 1) mask |= 1 << comp;
        }
        zero_rows(c, tlim::kTgtVisc, tlim::kTgtVisc + 3);
        tlim::launch_gershgorin_visc(c->stream, g0, o->face_mean, c->Lam, c->rC, wc, mask, row(c, tlim::kTgtVisc));
        tlim_status st = read_result(c, tlim::kTgtVisc, tlim::kTgtVisc + 3);
        if (st) return st;
        for (int comp = 0; comp < 3; ++comp) lam_c[comp] = result(c, tlim::kTgtVisc + comp);
    }
    for (int comp = 0; comp < 3; ++comp) {
        if (c->n[comp] <= 1) continue;
        double scale[3] = {1.0, 1.0, 1.0};
        scale[comp] = 4.0 / 3.0;
        DevGrid g = dev_grid(c, scale);
        const double lam = o->frozen_visc ? o->frozen_visc[comp] : lam_c[comp];
        PassSchedule ps = host_schedule(o->dt, lam, o->order);
        double* u = c->field[TLIM_U + comp];
        Vhat vh;
        tm.skip = true;  // the viscous passes are left out of the sweep timing
        run_lim_pass(c, g, o->face_mean, o->dt, ps, u, u, c->Tnew, nullptr, tlim::PassSlots{}, tm, sc, false,
                     heat || E ? &vh : nullptr);
        if (heat || E)
            tlim::launch_visc_heat(c->stream, g, ph, o->alpha_eps, o->face_mean, o->dt, c->field[TLIM_ALPHA2],
                                   c->field[TLIM_M1], c->field[TLIM_M2], c->Lam, vh.v64, vh.g64, vh.w32,
                                   heat ? c->field[TLIM_T1] : nullptr, heat ? c->field[TLIM_T2] : nullptr, E);
        std::swap(c->field[TLIM_U + comp], c->Tnew);
        if (rep) {
            rep->visc_P[comp] = lim_P(o->dt, lam);
            rep->visc_lambda_G[comp] = lam;
        }
    }
    return TLIM_OK;
}

// Heat-conduction coefficients of pass `it` at the current iterate (T1,
// alpha2) and the Gershgorin bound (max into *lam); sets c->g_heat.
bool fast_coeffs(const tlim_ctx* c, const DevGrid& g) {
    return !(c->fset[TLIM_SRC1] || c->fset[TLIM_SRC2]) && tlim::coeffs2d_applies(g);
}

void heat_coeffs(tlim_ctx* c, const DevGrid& g, const DevPhases& ph, const tlim_step_opts* o, double* lam, int it) {
    // T^(0) is the relaxed state T^n
    const double* T = it == 0 ? c->Tn : c->field[TLIM_T1];
    if (fast_coeffs(c, g)) {
        // 1/C depends on T only through B1 = p_inf,1 - p_inf,2
        const bool rebuild = it == 0 || c->phase[0].pinf != c->phase[1].pinf;
        const bool need_lam64 = c->precision == TLIM_FP64 || o->cycle_mode;
        tlim::launch_coeffs2d(c->stream, g, ph, o->alpha_eps, o->dt, o->face_mean, T, c->field[TLIM_ALPHA2],
                              c->field[TLIM_M1], c->field[TLIM_M2], c->Tn, rebuild ? 1 : 0,
                              need_lam64 ? c->Lam : nullptr, c->rC, c->Lam32, c->rC32, c->q32, nullptr, lam);
        c->g_heat = c->Tn;
        c->w0_zero = true;
        return;
    }
    tlim::launch_heat_coeffs_bound(c->stream, g, ph, o->alpha_eps, o->dt, o->face_mean, T, c->field[TLIM_ALPHA2],
                                   c->field[TLIM_M1], c->field[TLIM_M2], c->Tn,
                                   c->fset[TLIM_SRC1] ? c->field[TLIM_SRC1] : nullptr,
                                   c->fset[TLIM_SRC2] ? c->field[TLIM_SRC2] : nullptr, c->Lam, c->rC, c->rhs,
                                   c->Lam32, c->rC32, c->q32, c->wb[0], lam);
    c->g_heat = c->rhs;
    c->w0_zero = false;
}

// Chebyshev cycles to the backward-Euler solution of one pass (cycle mode).
tlim_status cycle_pass(tlim_ctx* c, const DevGrid& g, const tlim_step_opts* o, int s_stages, double lam,
                       int* cycles, double* residual, Timer& tm, SweepCount& sc) {
    std::vector<double> b = cycle_params(s_stages, lam);
    tlim::launch_copy(c->stream, c->vb[0], c->Tn, c->N);
    int cur = 0;
    int cyc = 0;
    double r = 0.0;
    tm.skip = true;  // every cycle follows the residual's readback: not timed
    while (cyc < o->max_cycles) {
        tm.start();
        for (int m = 0; m < s_stages; ++m) {
            tlim::StageParam sp{nullptr, o->dt * b[m], 0.0};
            tlim::launch_stage64(c->stream, g, o->face_mean, c->vb[cur], c->g_heat, c->Lam, c->rC, c->vb[cur ^ 1],
                                 sp, o->dt);
            cur ^= 1;
            sc.launches++;
        }
        tm.stop();
        sc.sweeps += s_stages;
        ++cyc;
        zero_rows(c, tlim::kTgtRR, tlim::kTgtGG + 1);
        tlim::launch_be_residual(c->stream, g, o->face_mean, c->vb[cur], c->g_heat, c->Lam, c->rC, o->dt,
                                 row(c, tlim::kTgtRR), row(c, tlim::kTgtGG));
        tlim_status st = read_result(c, tlim::kTgtRR, tlim::kTgtGG + 1);
        if (st) return st;
        double rr = result(c, tlim::kTgtRR), gg = result(c, tlim::kTgtGG);
        r = gg > 0.0 ? std::sqrt(rr / gg) : std::sqrt(rr);
        if (r < o->cycle_tol) break;
    }
    tlim::launch_copy(c->stream, c->Tnew, c->vb[cur], c->N);
    *cycles = cyc;
    *residual = r;
    return TLIM_OK;
}

enum class Mode { Sync, Frozen, Predict };

struct HeatOutcome {
    int passes_run = 0;
    bool converged = false;
    bool cycle_fail = false;
    bool mispredicted = false;
    double last_err = 0.0;
    double bad = 0.0;
};

// Picard loop of Algorithm 1 from the relaxed state (T1 = T^n, copied in Tn).
// Sync: one readback per pass brings lambda_G of the pass (and the change of
// the previous one).  Frozen: lambda per pass from the caller.  Predict: the
// P of each pass is taken from the previous step and the stages read lambda_G
// from device memory; the predictions are checked after one readback at the
// end (mispredicted = true means the caller must roll back and rerun).
// After a verified step with lambda_G per pass lam[0..passes), predict P of
// every pass of the next step.  Its first pass starts from T^{n+1}, the
// output of this step's last pass, whose conductivities are closest to this
// step's last lagged iterate: it gets the bound of this step's last pass.
// Its later passes follow the same pass of this step, extrapolated with the
// change since the step before when that change is small (the bound drifts
// as T smooths; a jump, e.g. from new material constants, is not a trend).
void record_schedule(tlim_ctx* c, int passes, const double* lam, double dt) {
    bool steady = c->hist_passes == passes;
    for (int i = 0; i < passes && steady; ++i) steady = lim_P(dt, lam[i]) == c->hist_P[i];
    c->hist_steady = steady ? c->hist_steady + 1 : 0;
    const bool have_prev = c->hist_nlam >= 1 && c->hist_passes == passes;
    for (int i = 0; i < passes; ++i) {
        double l = i == 0 ? lam[passes - 1] : lam[i];
        if (i > 0 && have_prev) {
            const double d = lam[i] - c->hist_lam[i];
            if (std::fabs(d) <= 0.1 * lam[i]) l += d;
        }
        c->hist_P[i] = lim_P(dt, l > 0.0 ? l : 0.0);
    }
    for (int i = 0; i < passes; ++i) c->hist_lam[i] = lam[i];
    c->hist_nlam = 1;
    c->hist_passes = passes;
}

// The blocked FP64 sweep can build the next pass's coefficients in its last
// launch: 2D grids without sources (conductivities from T and alpha2 only)
// and equal p_inf (1/C and alpha2 fixed within the step).
bool next_coef_ok(const tlim_ctx* c, const DevGrid& g) {
    return fast_coeffs(c, g) && g.nz == 1 && c->phase[0].pinf == c->phase[1].pinf;
}

// After a pass whose last launch built the next pass's coefficients.
void adopt_next_coef(tlim_ctx* c) {
    if (c->precision == TLIM_FP32) {
        std::swap(c->Lam32, c->Lam32_alt);
        std::swap(c->q32, c->q32_alt);
        c->w0_zero = true;
    } else {
        std::swap(c->Lam, c->Lam_alt);
    }
}

tlim::NextCoef next_coef(tlim_ctx* c, int it, const DevPhases& ph) {
    tlim::NextCoef nc{};
    nc.lam = row(c, tlim::tgt_lam(it + 1));
    nc.alpha2 = c->field[TLIM_ALPHA2];
    nc.Lam = c->Lam_alt;
    nc.Lam32 = c->Lam32_alt;
    nc.q32 = c->q32_alt;
    nc.ph = ph;
    nc.m1 = c->field[TLIM_M1];
    nc.m2 = c->field[TLIM_M2];
    return nc;
}

// A T^n array that neither the current step nor a pending (unverified)
// one uses.
double* free_tn(const tlim_ctx* c) {
    for (double* b : c->Tn_buf)
        if (b != c->Tn && !(c->pending && b == c->pend.Tn)) return b;
    return nullptr;  // unreachable: three arrays, at most two in use
}

// An alpha2 array (a2n or a2x, never the field) that a pending step does
// not need for a redo.
double* free_alpha2(const tlim_ctx* c) {
    return c->pending && c->a2n == c->pend.alpha2 ? c->a2x : c->a2n;
}

// The last launch of an FP64 step without sources and with equal p_inf can
// also relax the next step's state and build its first coefficients (what
// the next step's relaxation kernel would compute from the same fields), as
// long as nothing changes the state in between.
bool next_step_ok(const tlim_ctx* c, const tlim_step_opts* o, const DevGrid& g) {
    // FP32 contexts: the relaxation in the launch that also runs the double
    // final stage costs about what the separate relaxation kernel does
    return c->precision == TLIM_FP64 && next_coef_ok(c, g) && !o->cycle_mode && o->picard_tol <= 0.0;
}

tlim::NextCoef next_step_coef(tlim_ctx* c, const tlim_step_opts* o, const DevPhases& ph) {
    if (!c->spare_clean) zero_rows(c, tlim::kTgtNextStep, tlim::kTgtNextStep + 1);
    c->spare_clean = false;
    tlim::NextCoef nc{};
    nc.lam = row(c, tlim::kTgtNextStep);
    nc.alpha2 = c->field[TLIM_ALPHA2];
    nc.Lam = c->Lam_alt;
    nc.Lam32 = c->Lam32_alt;
    nc.q32 = c->q32_alt;
    nc.ph = ph;
    nc.m1 = c->field[TLIM_M1];
    nc.m2 = c->field[TLIM_M2];
    nc.next_step = 1;
    nc.Tn = c->next_tn = free_tn(c);  // the next step's T^n array
    nc.a2 = c->next_a2 = free_alpha2(c);
    nc.eps = o->alpha_eps;
    return nc;
}

// After the last launch of a step: whether it built the next step's start.
void note_next_step(tlim_ctx* c, const tlim_step_opts* o, bool done) {
    c->next_ready = done;
    c->next_eps = o->alpha_eps;
}

// pass0_done: the coefficients and bound of the first pass were built with
// the relaxation (and the accumulator rows zeroed before it).
tlim_status heat_passes(tlim_ctx* c, const tlim_step_opts* o, Mode mode, tlim_step_report* rep, Timer& tm,
                        SweepCount& sc, HeatOutcome& out, bool pass0_done) {
    hipStream_t s = c->stream;
    DevGrid g = dev_grid(c, kUnit);
    DevPhases ph = dev_phases(c);
    const bool B1 = c->phase[0].pinf != c->phase[1].pinf;
    int it;
    int P_used[TLIM_MAX_PASSES] = {0};
    if (!pass0_done) begin_pass_rows(c, o->passes);
    auto change = [&](int i) {
        double tmax = result(c, tlim::tgt_tmax(i)), dmax = result(c, tlim::tgt_dmax(i));
        return tmax > 0.0 ? dmax / tmax : dmax;
    };
    bool coef_ready = pass0_done;  // this pass's coefficients were built by the step before it
    for (it = 0; it < o->passes; ++it) {
        if (!coef_ready) heat_coeffs(c, g, ph, o, row(c, tlim::tgt_lam(it)), it);
        coef_ready = false;
        // previous iterate T^(it) (T^(0) = T^n)
        const double* Tit = it == 0 ? c->Tn : c->field[TLIM_T1];
        double lam = 0.0;
        if (mode == Mode::Sync) {
            // one readback: lambda_G of this pass and the change of the previous one
            tlim_status st = read_result(c, tlim::tgt_lam(0), tlim::tgt_lam(it + 1));
            if (st) return st;
            lam = result(c, tlim::tgt_lam(it));
            if (it > 0) {
                out.last_err = change(it - 1);
                if (rep) rep->err[it - 1] = out.last_err;
                if (o->picard_tol > 0.0 && out.last_err < o->picard_tol) {
                    out.converged = true;
                    out.bad = result(c, tlim::tgt_bad(it - 1));
                    break;
                }
            }
        } else if (mode == Mode::Frozen) {
            lam = o->frozen_lambda[it];
        }
        PassSchedule ps;
        int P;
        if (mode == Mode::Predict) {
            P = c->hist_P[it];
            ps = device_schedule(P, o->order, row(c, tlim::tgt_lam(it)));
        } else {
            P = lim_P(o->dt, lam);
            ps = host_schedule(o->dt, lam, o->order);
            if (rep) rep->lambda_G[it] = lam;
        }
        P_used[it] = P;
        if (rep) rep->P[it] = P;
        const bool need_update = B1 || o->cycle_mode;
        if (o->cycle_mode) {
            int ncyc = 0;
            double res = 0.0;
            tlim_status st = cycle_pass(c, g, o, 2 * P - 1, lam, &ncyc, &res, tm, sc);
            if (st) return st;
            if (rep) {
                rep->cycles[it] = ncyc;
                rep->residual[it] = res;
            }
            if (!(res < o->cycle_tol)) out.cycle_fail = true;  // keep the last iterate
        } else {
            const bool last = it + 1 == o->passes;
            const bool want = !need_update && !last && next_coef_ok(c, g);
            const bool want_step = !need_update && last && next_step_ok(c, o, g);
            tlim::NextCoef nc = want_step ? next_step_coef(c, o, ph) : next_coef(c, it, ph);
            bool done = false;
            // timed only behind the step's earlier passes (not after a readback)
            tm.skip = mode == Mode::Sync || it == 0;
            run_lim_pass(c, g, o->face_mean, o->dt, ps, c->Tn, c->g_heat, c->Tnew, need_update ? nullptr : Tit,
                         pass_slots(c, it, rep != nullptr || o->picard_tol > 0.0), tm, sc, true, nullptr,
                         want || want_step ? &nc : nullptr, &done);
            if (want_step) note_next_step(c, o, done);
            else if (done) {
                coef_ready = true;
                adopt_next_coef(c);
            }
        }
        if (need_update) {
            tlim::launch_pass_update(s, g, ph, o->alpha_eps, Tit, c->Tnew, c->Tn, c->a2n,
                                     c->field[TLIM_ALPHA2], c->field[TLIM_M1], c->field[TLIM_M2],
                                     c->field[TLIM_ALPHA2], pass_slots(c, it));
        }
        std::swap(c->field[TLIM_T1], c->Tnew);
    }
    out.passes_run = it;
    if (!out.converged) {
        // it = o->passes here: the readback consumes every row the step used
        // the next step's first bound, if this step's last launch built it,
        // moves into the first pass's row with the same fold
        const bool move = c->next_ready;
        tlim_status st = read_result(c, tlim::tgt_lam(0), tlim::tgt_lam(it), true, move ? tlim::kTgtNextStep : -1);
        if (st) return st;
        c->clean_rows = c->clean_keep;
        if (move) {
            c->row0_moved = true;
            c->spare_clean = true;
        }
        int last = it - 1;
        out.last_err = change(last);
        out.bad = result(c, tlim::tgt_bad(last));
        if (rep) rep->err[last] = out.last_err;
        if (o->picard_tol > 0.0 && out.last_err < o->picard_tol) out.converged = true;
    }
    if (mode == Mode::Predict) {
        // check every predicted P against the bound the step actually met
        for (int i = 0; i < out.passes_run; ++i) {
            double lam = result(c, tlim::tgt_lam(i));
            if (rep) rep->lambda_G[i] = lam;
            if (lim_P(o->dt, lam) != P_used[i]) out.mispredicted = true;
        }
        if (rep)
            for (int i = 0; i + 1 < out.passes_run; ++i) rep->err[i] = change(i);
    }
    if (mode != Mode::Frozen && !out.mispredicted && !o->cycle_mode && out.passes_run > 0) {
        // The next step's passes start from T^{n+1}, the output of this step's
        // last pass, whose conductivities are closest to this step's last
        // lagged iterate: predict every pass of the next step with the P of
        // this step's last pass.
        double lv[TLIM_MAX_PASSES];
        for (int i = 0; i < out.passes_run; ++i) lv[i] = result(c, tlim::tgt_lam(i));
        record_schedule(c, out.passes_run, lv, o->dt);
    } else {
        c->hist_steady = 0;
    }
    return TLIM_OK;
}

}  // namespace

// =================================================================== C ABI

namespace tlim {

DevPhases pack_phases(const tlim_phase ph[2]) {
    DevPhases p{};
    for (int k = 0; k < 2; ++k) {
        p.gamma[k] = ph[k].gamma;
        p.pinf[k] = ph[k].pinf;
        p.cv[k] = ph[k].cv;
        p.qf[k] = ph[k].q;
        p.k0[k] = ph[k].k0;
        p.T0[k] = ph[k].T0;
        p.invT0[k] = 1.0 / ph[k].T0;
        p.npow[k] = ph[k].npow;
        p.mu[k] = ph[k].mu;
        p.sh_law[k] = ph[k].law == TLIM_LAW_SPITZER;
        if (p.sh_law[k]) {
            p.spitzer = 1;
            p.ln_shD[k] = std::log(ph[k].sh_D);
            p.ln_shLD[k] = std::log(ph[k].sh_LD);  // -inf for 0: that length never wins
            p.ln_shdB[k] = std::log(ph[k].sh_dB);
        }
    }
    return p;
}

DevGrid pack_grid(const tlim_grid* gr) {
    DevGrid g{};
    g.nx = (int)gr->n[0];
    g.ny = (int)gr->n[1];
    g.nz = (int)gr->n[2];
    for (int d = 0; d < 3; ++d) {
        g.per[d] = gr->bc[d] == TLIM_PERIODIC;
        g.w[d] = 1.0 / (gr->h[d] * gr->h[d]);
    }
    g.N = gr->n[0] * gr->n[1] * gr->n[2];
    return g;
}

const char* check_grid(const tlim_grid* g) {
    if (!g) return "grid is NULL";
    // launch limits of the tiled kernels: ceil(ny/4) and nz blocks along y and z
    const int64_t nmax[3] = {(int64_t)1 << 24, (int64_t)4 * 65535, 65535};
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 1 || g->n[d] > nmax[d]) return "cell count out of range on an axis";
        if (!(g->h[d] > 0.0) || !std::isfinite(g->h[d])) return "spacing must be finite and > 0";
        if (g->bc[d] != TLIM_PERIODIC && g->bc[d] != TLIM_ADIABATIC) return "unknown boundary condition";
    }
    if (g->n[0] * g->n[1] * g->n[2] > ((int64_t)1 << 34)) return "more than 2^34 cells";
    return nullptr;
}

const char* check_phase(const tlim_phase* p) {
    if (!p) return "phase is NULL";
    if (!(p->gamma > 1.0) || !(p->cv > 0.0) || !(p->k0 >= 0.0) || !(p->T0 > 0.0) || !(p->mu >= 0.0) ||
        !std::isfinite(p->pinf) || !std::isfinite(p->npow))
        return "invalid phase constants";
    if (p->law != TLIM_LAW_POWER && p->law != TLIM_LAW_SPITZER) return "unknown conductivity law";
    if (p->law == TLIM_LAW_SPITZER &&
        (!(p->sh_D > 0.0) || !(p->sh_LD >= 0.0) || !(p->sh_dB >= 0.0) || !(p->sh_LD > 0.0 || p->sh_dB > 0.0) ||
         !std::isfinite(p->sh_D) || !std::isfinite(p->sh_LD) || !std::isfinite(p->sh_dB)))
        return "invalid Spitzer-Harm length constants";
    return nullptr;
}

namespace {
thread_local std::string free_error;
}

void set_free_error(const char* msg) { free_error = msg ? msg : ""; }

}  // namespace tlim

extern "C" {

namespace {
tlim_status resolve(tlim_ctx* c);
}  // namespace


const char* tlim_status_str(tlim_status s) {
    switch (s) {
        case TLIM_OK: return "TLIM_OK";
        case TLIM_E_ARG: return "TLIM_E_ARG";
        case TLIM_E_STATE: return "TLIM_E_STATE";
        case TLIM_E_HIP: return "TLIM_E_HIP";
        case TLIM_E_NOMEM: return "TLIM_E_NOMEM";
        case TLIM_E_NOCONV: return "TLIM_E_NOCONV";
        case TLIM_E_NUMERIC: return "TLIM_E_NUMERIC";
    }
    return "unknown";
}

const char* tlim_last_error(const tlim_ctx* c) { return c ? c->err.c_str() : tlim::free_error.c_str(); }

tlim_status tlim_create(const tlim_grid* grid, int32_t precision, void* hip_stream, tlim_ctx** out) {
    if (!grid || !out) return TLIM_E_ARG;
    *out = nullptr;
    if (tlim::check_grid(grid)) return TLIM_E_ARG;
    if (precision != TLIM_FP64 && precision != TLIM_FP32) return TLIM_E_ARG;
    int64_t N = grid->n[0] * grid->n[1] * grid->n[2];
    tlim_ctx* c = new tlim_ctx();
    for (int d = 0; d < 3; ++d) {
        c->n[d] = grid->n[d];
        c->h[d] = grid->h[d];
        c->bc[d] = grid->bc[d];
    }
    c->N = N;
    c->precision = precision;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return TLIM_E_HIP;
    }
    // coherent: a fold's stores reach the host while later kernels run (the
    // readbacks poll its sequence number, not an event).  Where only the
    // default kind exists, the polls end in their stream drain instead.
    if (hipHostMalloc((void**)&c->res_blk[0], 2 * sizeof(PassResult), hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        if (hipHostMalloc((void**)&c->res_blk[0], 2 * sizeof(PassResult), hipHostMallocDefault) != hipSuccess) {
            delete c;
            return TLIM_E_HIP;
        }
    }
    c->res_blk[1] = c->res_blk[0] + 1;
    if (hipHostGetDevicePointer((void**)&c->res_blk_dev[0], c->res_blk[0], 0) != hipSuccess) {
        c->res_blk_dev[0] = nullptr;
        (void)hipGetLastError();
    }
    c->res_blk_dev[1] = c->res_blk_dev[0] ? c->res_blk_dev[0] + 1 : nullptr;
    c->res_blk[0]->seq = c->res_blk[1]->seq = 0;
    c->res_seq = 0;
    c->res_cur = 0;
    c->res_host = c->res_blk[0];
    c->res_host_dev = c->res_blk_dev[0];
    c->clean_rows = c->clean_keep = 0;
    c->pending = false;
    c->step2d_spin_limit = 1u << 20;
    if (const char* e = std::getenv("TLIM_STEP2D_SPIN_LIMIT")) {
        // test hook: a small limit forces the time-out path from the host
        char* end = nullptr;
        const unsigned long v = std::strtoul(e, &end, 10);
        if (end != e && v <= 0xffffffffUL) c->step2d_spin_limit = (unsigned)v;
    }
    for (int i = 0; i < kMaxEvents; ++i) {
        if (hipEventCreate(&c->ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->ev[j]);
            (void)hipHostFree(c->res_blk[0]);
            delete c;
            return TLIM_E_HIP;
        }
    }
    if (hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_pend[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_pend[1], hipEventDisableTiming) != hipSuccess) {
        for (int j = 0; j < kMaxEvents; ++j) (void)hipEventDestroy(c->ev[j]);
        (void)hipHostFree(c->res_blk[0]);
        delete c;
        return TLIM_E_HIP;
    }
    *out = c;
    return TLIM_OK;
}

tlim_status tlim_destroy(tlim_ctx* c) {
    if (!c) return TLIM_OK;
    (void)resolve(c);
    for (int i = 0; i < kMaxEvents; ++i) (void)hipEventDestroy(c->ev[i]);
    (void)hipEventDestroy(c->ev_sync);
    (void)hipEventDestroy(c->ev_pend[0]);
    (void)hipEventDestroy(c->ev_pend[1]);
    (void)hipHostFree(c->res_blk[0]);
    delete c;
    return TLIM_OK;
}

tlim_status tlim_workspace_bytes(const tlim_ctx* c, size_t* bytes) {
    if (!c || !bytes) return TLIM_E_ARG;
    *bytes = layout_of(c->n, c->precision).total;
    return TLIM_OK;
}

tlim_status tlim_bind_workspace(tlim_ctx* c, void* dev_ptr, size_t bytes) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    if (!dev_ptr || ((uintptr_t)dev_ptr % kAlign) != 0) return fail(c, TLIM_E_ARG, "workspace NULL or not 256-byte aligned");
    Layout L = layout_of(c->n, c->precision);
    if (bytes < L.total) return fail(c, TLIM_E_NOMEM, "workspace %zu bytes < %zu required", bytes, L.total);
    char* base = (char*)dev_ptr;
    c->ws = base;
    c->ws_bytes = bytes;
    for (int i = 0; i < TLIM_NFIELDS; ++i) {
        c->field[i] = (double*)(base + L.field[i]);
        c->fset[i] = false;
    }
    c->Tn = (double*)(base + L.Tn);
    c->Tn_buf[0] = c->Tn;
    c->Tn_buf[1] = (double*)(base + L.Tn2);
    c->Tn_buf[2] = (double*)(base + L.Tn3);
    c->a2x = (double*)(base + L.a2x);
    c->Tnew = (double*)(base + L.Tnew);
    c->a2n = (double*)(base + L.a2n);
    c->a2pool[0] = c->field[TLIM_ALPHA2];
    c->a2pool[1] = c->a2n;
    c->a2pool[2] = c->a2x;
    c->Lam = (double*)(base + L.Lam);
    c->Lam_alt = (double*)(base + L.Lam2);
    c->rC = (double*)(base + L.rC);
    c->next_ready = false;
    c->spare_clean = true;  // zeroed below
    c->row0_moved = false;
    c->rhs = (double*)(base + L.rhs);
    c->vb[0] = (double*)(base + L.vb[0]);
    c->vb[1] = (double*)(base + L.vb[1]);
    c->acc = (double*)(base + L.acc);
    c->res_dev = (PassResult*)(base + L.res);
    c->chat_tab = (double*)(base + L.chat);
    c->chat_order = -1;
    c->bar = (unsigned*)(base + L.bar);
    c->collect_done = (unsigned*)(base + L.cnt);
    tlim::launch_fill(c->stream, (double*)c->collect_done, 0.0, 1);
    c->t2_alias = false;
    c->hist_passes = 0;
    c->hist_steady = 0;
    c->hist_nlam = 0;
    c->clean_rows = c->clean_keep = 0;  // the new accumulator is not known to be zero
    zero_rows(c, tlim::kTgtFlag, tlim::kTgtNextStep + 1);
    if (c->precision == TLIM_FP32) {
        c->Lam32 = (float*)(base + L.Lam32);
        c->rC32 = (float*)(base + L.rC32);
        c->q32 = (float*)(base + L.q32);
        c->wb[0] = (float*)(base + L.wb[0]);
        c->wb[1] = (float*)(base + L.wb[1]);
        c->Lam32_alt = (float*)(base + L.Lam32b);
        c->q32_alt = (float*)(base + L.q32b);
        c->wzero = (float*)(base + L.wzero);
        HIP_TRY(c, hipMemsetAsync(c->wzero, 0, sizeof(float) * (size_t)c->N, c->stream));
    } else {
        c->Lam32 = c->rC32 = c->q32 = c->wb[0] = c->wb[1] = nullptr;
        c->Lam32_alt = c->q32_alt = c->wzero = nullptr;
    }
    c->w0_zero = false;
    return step2d_table(c, TLIM_ORDER_INTERLEAVED);
}

tlim_status tlim_set_phase(tlim_ctx* c, int32_t k, const tlim_phase* p) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    c->next_ready = false;  // the state or the laws change
    if (k < 0 || k > 1 || !p) return fail(c, TLIM_E_ARG, "phase index must be 0 or 1");
    if (const char* why = tlim::check_phase(p)) return fail(c, TLIM_E_ARG, "%s", why);
    c->phase[k] = *p;
    c->phase_set[k] = true;
    return TLIM_OK;
}

tlim_status tlim_set_field(tlim_ctx* c, int32_t f, const void* src, int32_t dtype) {
    if (!c) return TLIM_E_ARG;
    if (f < 0 || f >= TLIM_NFIELDS || !src) return fail(c, TLIM_E_ARG, "bad field index or NULL source");
    if (dtype != TLIM_DTYPE_F64 && dtype != TLIM_DTYPE_F32) return fail(c, TLIM_E_ARG, "unknown dtype %d", dtype);
    tlim_status pst = resolve(c);
    if (pst) return pst;
    c->next_ready = false;  // the state or the laws change
    if (!c->ws) return fail(c, TLIM_E_STATE, "no workspace bound");
    if (c->t2_alias && (f == TLIM_T1 || f == TLIM_T2)) {
        // give T2 its own values again before either temperature changes
        tlim::launch_copy(c->stream, c->field[TLIM_T2], c->field[TLIM_T1], c->N);
        c->t2_alias = false;
    }
    if (dtype == TLIM_DTYPE_F64)
        HIP_TRY(c, hipMemcpyAsync(c->field[f], src, sizeof(double) * (size_t)c->N, hipMemcpyDeviceToDevice, c->stream));
    else
        tlim::launch_widen(c->stream, c->field[f], (const float*)src, c->N);
    c->fset[f] = true;
    return TLIM_OK;
}

tlim_status tlim_get_field(tlim_ctx* c, int32_t f, void* dst, int32_t dtype) {
    if (!c) return TLIM_E_ARG;
    if (f < 0 || f >= TLIM_NFIELDS || !dst) return fail(c, TLIM_E_ARG, "bad field index or NULL destination");
    if (dtype != TLIM_DTYPE_F64 && dtype != TLIM_DTYPE_F32) return fail(c, TLIM_E_ARG, "unknown dtype %d", dtype);
    tlim_status pst = resolve(c);
    if (pst) return pst;
    if (!c->ws || !c->fset[f]) return fail(c, TLIM_E_STATE, "field %d not set", f);
    const double* src = f == TLIM_T2 ? T2_ptr(c) : c->field[f];
    if (dtype == TLIM_DTYPE_F64)
        HIP_TRY(c, hipMemcpyAsync(dst, src, sizeof(double) * (size_t)c->N, hipMemcpyDeviceToDevice, c->stream));
    else
        tlim::launch_narrow(c->stream, (float*)dst, src, c->N);
    return TLIM_OK;
}

tlim_status tlim_clear_field(tlim_ctx* c, int32_t f) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    c->next_ready = false;  // the state or the laws change
    if (f < TLIM_U || f >= TLIM_NFIELDS) return fail(c, TLIM_E_ARG, "field %d is not optional", f);
    c->fset[f] = false;
    return TLIM_OK;
}

// ---- hyperbolic part and pressure relaxation (Sec. 3.1, Sec. 3.3)

tlim_status tlim_advance_hyperbolic(tlim_ctx* c, const tlim_hyp_opts* o, tlim_hyp_report* rep) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    c->next_ready = false;  // the state changes
    if (!o || !(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(c, TLIM_E_ARG, "dt must be finite and > 0");
    tlim_status st = check_ready(c);
    if (st) return st;
    hipStream_t s = c->stream;
    if (c->t2_alias) {
        tlim::launch_copy(s, c->field[TLIM_T2], c->field[TLIM_T1], c->N);
        c->t2_alias = false;
    }
    const DevGrid g = dev_grid(c, kUnit);
    const DevPhases ph = dev_phases(c);
    // the state's fields in the order of the conservative components; the
    // velocity components and rho E that are not set count as zero and as
    // the energy of the state
    const int fidx[9] = {TLIM_M1, TLIM_M2, TLIM_U, TLIM_V, TLIM_W, TLIM_T1, TLIM_T2, TLIM_E, TLIM_ALPHA2};
    double* F[9];
    const double* prim[9];
    for (int k = 0; k < 9; ++k) {
        F[k] = c->field[fidx[k]];
        prim[k] = c->fset[fidx[k]] ? F[k] : nullptr;
    }
    // U ping-pongs between scratch arrays (free between steps) and the field
    // storage so that the last sweep writes the fields.  With an even number
    // of sweeps the first one reads the state itself and converts it on
    // load; otherwise U is built in the scratch arrays first.
    double* A[9] = {c->Tn_buf[0], c->Tn_buf[1], c->Tn_buf[2], c->Tnew, c->a2n, c->a2x, c->Lam, c->Lam_alt, c->rC};
    int axes[3], ns = 0;
    for (int d = 0; d < 3; ++d)
        if (c->n[d] > 1) axes[ns++] = d;
    double* bad = row(c, tlim::kTgtHypBad);
    zero_rows(c, tlim::kTgtHypBad, tlim::kTgtHypBad + 1);
    const bool fused = ns % 2 == 0 && ns > 0;
    if (!fused) tlim::launch_hyp_cons(s, g, ph, prim, A);
    if (ns == 0) {
        tlim::launch_hyp_sweep(s, g, ph, 0, 0.0, 0, A, F, 0, 1, bad);  // no face: back to the fields
    } else {
        double* const* cur = fused ? F : A;
        for (int k = 0; k < ns; ++k) {
            const int d = axes[k];
            double* const* out = cur == A ? F : A;
            const bool first = k == 0 && fused;
            tlim::launch_hyp_sweep(s, g, ph, d, o->dt / c->h[d], o->relax_pressure ? 1 : 0,
                                   first ? prim : (const double* const*)cur, out, first ? 1 : 0,
                                   k == ns - 1 ? 1 : 0, bad);
            cur = out;
        }
    }
    HIP_TRY(c, hipGetLastError());
    for (int f : {TLIM_U, TLIM_V, TLIM_W, TLIM_E}) c->fset[f] = true;
    if (rep) {
        st = read_result(c, tlim::kTgtHypBad, tlim::kTgtHypBad + 1);
        if (st) return st;
        rep->bad_cells = result(c, tlim::kTgtHypBad);
        if (rep->bad_cells > 0.0)
            return fail(c, TLIM_E_NUMERIC, "%.0f cells left 0 < alpha2 < 1 or lost a positive temperature",
                        rep->bad_cells);
    }
    return TLIM_OK;
}

tlim_status tlim_hyperbolic_dt(tlim_ctx* c, double cfl, double* dt_out) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    if (!dt_out || !(cfl > 0.0) || !std::isfinite(cfl)) return fail(c, TLIM_E_ARG, "cfl must be finite and > 0");
    tlim_status st = check_ready(c);
    if (st) return st;
    const DevGrid g = dev_grid(c, kUnit);
    const DevPhases ph = dev_phases(c);
    const int fidx[9] = {TLIM_M1, TLIM_M2, TLIM_U, TLIM_V, TLIM_W, TLIM_T1, TLIM_T2, TLIM_E, TLIM_ALPHA2};
    const double* prim[9];
    for (int k = 0; k < 9; ++k) prim[k] = c->fset[fidx[k]] ? c->field[fidx[k]] : nullptr;
    prim[6] = T2_ptr(c);
    double ih[3];
    for (int d = 0; d < 3; ++d) ih[d] = c->n[d] > 1 ? 1.0 / c->h[d] : 0.0;
    zero_rows(c, tlim::kTgtHypRate, tlim::kTgtHypRate + 1);
    tlim::launch_hyp_rate(c->stream, g, ph, prim, ih, row(c, tlim::kTgtHypRate));
    st = read_result(c, tlim::kTgtHypRate, tlim::kTgtHypRate + 1);
    if (st) return st;
    const double rate = result(c, tlim::kTgtHypRate);
    *dt_out = rate > 0.0 ? cfl / rate : 0.0;
    return TLIM_OK;
}

tlim_status tlim_spectral_bound(tlim_ctx* c, int32_t face_mean, double alpha_eps, double* lambda_out) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    c->next_ready = false;  // the relaxation below uses the spare arrays
    if (!lambda_out || face_mean < 0 || face_mean > 1 || alpha_eps < 0.0 || alpha_eps >= 0.5)
        return fail(c, TLIM_E_ARG, "bad arguments");
    tlim_status st = check_ready(c);
    if (st) return st;
    // relax copies of (alpha2, T1, T2) into scratch, leaving the state untouched
    DevGrid g = dev_grid(c, kUnit);
    DevPhases ph = dev_phases(c);
    tlim::launch_copy(c->stream, c->a2n, c->field[TLIM_ALPHA2], c->N);
    tlim::launch_copy(c->stream, c->Tn, c->field[TLIM_T1], c->N);
    tlim::launch_copy(c->stream, c->Tnew, T2_ptr(c), c->N);
    tlim::launch_relax(c->stream, g, ph, alpha_eps, c->a2n, c->field[TLIM_M1], c->field[TLIM_M2], c->Tn, c->Tnew,
                       nullptr, nullptr);
    zero_rows(c, tlim::kTgtLambda, tlim::kTgtLambda + 1);
    tlim::launch_heat_coeffs_bound(c->stream, g, ph, alpha_eps, 1.0, face_mean, c->Tn, c->a2n, c->field[TLIM_M1],
                                   c->field[TLIM_M2], c->Tn, nullptr, nullptr, c->Lam, c->rC, c->rhs, nullptr,
                                   nullptr, nullptr, nullptr, row(c, tlim::kTgtLambda));
    st = read_result(c, tlim::kTgtLambda, tlim::kTgtLambda + 1);
    if (st) return st;
    *lambda_out = result(c, tlim::kTgtLambda);
    return TLIM_OK;
}

namespace {

// ---- whole-step kernel (2D, FP64, no sources, equal p_inf)

// The step runs as one cooperative launch (relaxation and every Picard pass,
// P decided on the device) when asked (always, or while there is no schedule
// history to predict P from), the grid's tiles can all be resident and the
// schedule is not given by the caller.
bool step2d_ok(const tlim_ctx* c, const tlim_step_opts* o) {
    // AUTO: the steps that would otherwise read each pass's bound back (no
    // schedule history, or one that has not yet held for a step)
    if (o->whole_step == TLIM_WHOLE_NEVER ||
        (o->whole_step == TLIM_WHOLE_AUTO && c->hist_passes == o->passes && c->hist_steady >= 1))
        return false;
    if (c->precision != TLIM_FP64 || o->cycle_mode || o->frozen_lambda || o->picard_tol > 0.0) return false;
    if (c->phase[0].pinf != c->phase[1].pinf) return false;
    const DevGrid g = dev_grid(c, kUnit);
    return fast_coeffs(c, g) && tlim::step2d_tiles(g) > 0;
}

// Enqueue a step by the whole-step kernel followed by the fold of its rows
// (lambda_G, change, bad cells, P per pass and the failure count) into `res`
// (device address of a pinned block; NULL: the device result block).  On
// success the relaxed state becomes the step's T^n and alpha2.  False: the
// launch was refused and nothing but the row clearing ran.
bool step2d_enqueue(tlim_ctx* c, const tlim_step_opts* o, PassResult* res) {
    hipStream_t s = c->stream;
    const DevGrid g = dev_grid(c, kUnit);
    begin_pass_rows(c, o->passes);
    tlim::launch_fill(s, (double*)c->bar, 0.0, tlim::kStepMaxTiles / 2);
    double* Tn = free_tn(c);
    tlim::Step2D st{};
    st.alpha2 = c->field[TLIM_ALPHA2];
    st.T1 = c->field[TLIM_T1];
    st.T2 = T2_ptr(c);
    st.m1 = c->field[TLIM_M1];
    st.m2 = c->field[TLIM_M2];
    st.Tn = Tn;
    st.a2n = c->a2n;
    st.rC = c->rC;
    // the last pass writes the T1 field (the relaxation has read it by then)
    const int f = (o->passes - 1) & 1;
    st.Tout[f] = c->field[TLIM_T1];
    st.Tout[1 - f] = c->Tnew;
    st.vx[0] = c->vb[0];
    st.vx[1] = c->vb[1];
    st.acc = c->acc;
    st.bar = c->bar;
    st.chat = c->chat_tab;
    st.pmax = kStepPmax;
    st.passes = o->passes;
    st.spin_limit = c->step2d_spin_limit;
    if (!tlim::launch_step2d(s, g, dev_phases(c), o->alpha_eps, o->dt, o->face_mean, st)) return false;
    c->next_ready = false;
    c->Tn = Tn;
    c->g_heat = Tn;
    std::swap(c->field[TLIM_ALPHA2], c->a2n);
    c->t2_alias = true;
    tlim::launch_collect(s, c->acc, res ? res : c->res_dev, tlim::tgt_lam(0), tlim::kTgtP0 + o->passes, 1);
    c->clean_rows = c->clean_keep;
    return true;
}

// Outcome of a whole-step run from its folded rows.  A failure count means
// a P beyond the table (rerun the passes from the relaxed state) or a
// barrier time-out.
struct Step2DResult {
    bool out_of_range = false, timeout = false;
    int P[TLIM_MAX_PASSES];
    double lam[TLIM_MAX_PASSES];
};
void step2d_result(const PassResult* r, int passes, Step2DResult& o) {
    o = Step2DResult{};
    for (int i = 0; i < passes; ++i) {
        o.lam[i] = r->v[tlim::tgt_lam(i)];
        const double P = r->v[tlim::kTgtP0 + i];
        o.P[i] = (int)P;
        if (r->v[tlim::kTgtFlag] > 0.0 && !(P >= 1.0 && P <= kStepPmax)) o.out_of_range = true;
    }
    if (r->v[tlim::kTgtFlag] > 0.0 && !o.out_of_range) o.timeout = true;
}

// One step's heat part by the whole-step kernel with a readback; on return
// `done` tells whether it ran (else the caller takes the launch-per-stage
// path from the unrelaxed state).
tlim_status step2d_sync(tlim_ctx* c, const tlim_step_opts* o, tlim_step_report* rep, Timer& tm, SweepCount& sc,
                        HeatOutcome& out, bool& done) {
    done = false;
    tlim_status st = step2d_table(c, o->order);
    if (st) return st;
    tm.skip = true;  // the step's first launch: not timed
    tm.start();
    const bool ok = step2d_enqueue(c, o, c->res_host_dev);
    tm.stop();
    tm.skip = false;
    if (!ok) return TLIM_OK;
    done = true;
    if (!c->res_host_dev) HIP_TRY(c, hipMemcpyAsync(c->res_host, c->res_dev, sizeof(PassResult), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    Step2DResult r;
    step2d_result(c->res_host, o->passes, r);
    if (r.timeout) return lose_heat_state(c);
    if (r.out_of_range) {
        // schedule beyond the table: the passes again, one launch per block of stages
        out = HeatOutcome{};
        return heat_passes(c, o, Mode::Sync, rep, tm, sc, out, false);
    }
    out.passes_run = o->passes;
    out.converged = true;
    auto change = [&](int i) {
        const double tmax = result(c, tlim::tgt_tmax(i)), dmax = result(c, tlim::tgt_dmax(i));
        return tmax > 0.0 ? dmax / tmax : dmax;
    };
    out.last_err = change(o->passes - 1);
    out.bad = result(c, tlim::tgt_bad(o->passes - 1));
    for (int i = 0; i < o->passes; ++i) {
        sc.sweeps += 2 * r.P[i] - 1;
        if (rep) {
            rep->P[i] = r.P[i];
            rep->lambda_G[i] = r.lam[i];
            rep->err[i] = change(i);
        }
    }
    sc.launches += 1;
    record_schedule(c, o->passes, r.lam, o->dt);
    return TLIM_OK;
}

// Temperature relaxation at the start of a step (Sec. 3.4.1).  On 2D grids
// without sources it is fused with the first pass's coefficients and bound
// (returns true); the relaxed state goes to Tn and a2n, and a2n becomes the
// alpha2 field.  T1 is not written: every pass starts from Tn and the last
// one writes T1.  T^n alternates between two arrays from step to step, so a
// step's T^n outlives the next step's enqueue.
bool relax_step(tlim_ctx* c, const tlim_step_opts* o) {
    hipStream_t s = c->stream;
    DevGrid g = dev_grid(c, kUnit);
    DevPhases ph = dev_phases(c);
    const bool B1 = c->phase[0].pinf != c->phase[1].pinf;
    bool pass0_done = false;
    if (c->next_ready && c->row0_moved && fast_coeffs(c, g) && !B1 && o->alpha_eps == c->next_eps) {
        // the previous step's last launch relaxed this state already: adopt
        // its relaxed T, alpha2 and Lambda (1/C is unchanged); its bound is in the first
        // pass's row, the other pass rows are zero up to clean_rows
        const int need = tlim::tgt_lam(o->passes);
        if (c->clean_rows < need) zero_rows(c, tlim::tgt_lam(1), need);
        c->clean_keep = std::max(c->clean_rows, need);
        c->clean_rows = 0;
        c->row0_moved = false;
        c->Tn = c->next_tn;
        double* old = c->field[TLIM_ALPHA2];
        c->field[TLIM_ALPHA2] = c->next_a2;
        if (c->a2n == c->next_a2) c->a2n = old;
        else c->a2x = old;
        adopt_next_coef(c);  // Lambda (FP32: float Lambda and the correction source)
        c->g_heat = c->Tn;
        c->next_ready = false;
        c->t2_alias = true;
        return true;
    }
    c->next_ready = false;
    c->Tn = free_tn(c);
    if (fast_coeffs(c, g)) {
        begin_pass_rows(c, o->passes);
        const bool need_lam64 = c->precision == TLIM_FP64 || o->cycle_mode;
        tlim::launch_coeffs2d(s, g, ph, o->alpha_eps, o->dt, o->face_mean, c->field[TLIM_T1], c->field[TLIM_ALPHA2],
                              c->field[TLIM_M1], c->field[TLIM_M2], nullptr, 1, need_lam64 ? c->Lam : nullptr, c->rC,
                              c->Lam32, c->rC32, c->q32, nullptr, row(c, tlim::tgt_lam(0)), T2_ptr(c), c->Tn,
                              c->a2n);
        c->w0_zero = true;
        std::swap(c->field[TLIM_ALPHA2], c->a2n);
        if (B1) tlim::launch_copy(s, c->a2n, c->field[TLIM_ALPHA2], c->N);  // kept for a rollback
        c->g_heat = c->Tn;
        pass0_done = true;
    } else {
        tlim::launch_relax(s, g, ph, o->alpha_eps, c->field[TLIM_ALPHA2], c->field[TLIM_M1], c->field[TLIM_M2],
                           c->field[TLIM_T1], T2_ptr(c), c->Tn, B1 ? c->a2n : nullptr);
    }
    c->t2_alias = true;  // T_1 = T_2 from here on
    return pass0_done;
}

// One step with a readback of its own (all modes).
tlim_status advance_sync(tlim_ctx* c, const tlim_step_opts* o, tlim_step_report* rep) {
    tlim_status st = TLIM_OK;
    if (rep) std::memset(rep, 0, sizeof(*rep));
    hipStream_t s = c->stream;
    DevGrid g = dev_grid(c, kUnit);
    DevPhases ph = dev_phases(c);
    const double vol = cell_volume(c);
    const bool B1 = c->phase[0].pinf != c->phase[1].pinf;
    Timer tm{c, o->time_sweeps != 0};
    SweepCount sc;

    if (rep) {
        zero_rows(c, tlim::kTgtEnergy, tlim::kTgtEnergy + 1);
        tlim::launch_energy(s, g, ph, c->field[TLIM_ALPHA2], c->field[TLIM_M1], c->field[TLIM_M2], c->field[TLIM_T1],
                            T2_ptr(c), row(c, tlim::kTgtEnergy));
        st = read_result(c, tlim::kTgtEnergy, tlim::kTgtEnergy + 1);
        if (st) return st;
        rep->energy_before = result(c, tlim::kTgtEnergy) * vol;
    }
    // splitting order of the paper: viscous part, temperature relaxation, heat conduction
    if (o->do_viscous) {
        st = viscous(c, o, rep, tm, sc);
        if (st) return st;
    }
    HeatOutcome out;
    bool whole = false;  // relaxation and passes by the whole-step kernel
    if (step2d_ok(c, o)) {
        st = step2d_sync(c, o, rep, tm, sc, out, whole);
        if (st) return st;
    }
    bool predicted = false, mispredicted = false;
    if (!whole) {
        const bool pass0_done = relax_step(c, o);
        Mode mode = Mode::Sync;
        if (o->frozen_lambda) mode = Mode::Frozen;
        // Predict only once the schedule has held for a step: a miss costs
        // the whole heat part twice, a readback per pass only a round trip
        // (where the first pass's bound keeps differing from the last pass's
        // of the step before, every prediction would miss)
        else if (!o->cycle_mode && o->picard_tol <= 0.0 && c->hist_passes == o->passes && c->hist_steady >= 1)
            mode = Mode::Predict;
        st = heat_passes(c, o, mode, rep, tm, sc, out, pass0_done);
        if (st) return st;
        predicted = mode == Mode::Predict && !out.mispredicted;
        mispredicted = out.mispredicted;
        if (out.mispredicted) {
            // roll back to the relaxed state and rerun with one readback per
            // pass; only the rerun's sweeps count
            c->predict_misses++;
            if (B1) tlim::launch_copy(s, c->field[TLIM_ALPHA2], c->a2n, c->N);
            out = HeatOutcome{};
            sc = SweepCount{};
            tm.reset();
            st = heat_passes(c, o, Mode::Sync, rep, tm, sc, out, false);
            if (st) return st;
        }
    }
    if (c->fset[TLIM_E]) tlim::launch_total_energy_heat(s, c->N, c->field[TLIM_T1], c->Tn, c->rC, c->field[TLIM_E]);
    if (rep) {
        zero_rows(c, tlim::kTgtEnergy, tlim::kTgtEnergy + 1);
        tlim::launch_energy(s, g, ph, c->field[TLIM_ALPHA2], c->field[TLIM_M1], c->field[TLIM_M2], c->field[TLIM_T1],
                            c->field[TLIM_T1], row(c, tlim::kTgtEnergy));
        st = read_result(c, tlim::kTgtEnergy, tlim::kTgtEnergy + 1);
        if (st) return st;
        rep->energy_after = result(c, tlim::kTgtEnergy) * vol;
        rep->passes_run = out.passes_run;
        rep->converged = (o->picard_tol <= 0.0 || out.converged) && !out.cycle_fail;
        rep->sweeps = sc.sweeps;
        rep->sweep_launches = sc.launches;
        rep->timed_sweeps = sc.timed_sweeps;
        rep->timed_launches = sc.timed_launches;
        rep->bad_cells = (int64_t)out.bad;
        rep->predicted = predicted ? 1 : 0;
        rep->mispredicted = mispredicted ? 1 : 0;
        rep->pipelined_steps = c->pipelined_steps;
        rep->pipeline_redos = c->pipeline_redos;
        if (tm.on) {
            HIP_TRY(c, hipStreamSynchronize(s));
            rep->sweep_ms = tm.elapsed_ms();
        }
    }
    HIP_TRY(c, hipGetLastError());
    if (out.bad > 0.0) return fail(c, TLIM_E_NUMERIC, "%.0f cells with non-finite or non-positive T", out.bad);
    if ((o->picard_tol > 0.0 && !out.converged) || out.cycle_fail)
        return fail(c, TLIM_E_NOCONV, "tolerance not reached (last Picard change %.3e)", out.last_err);
    return TLIM_OK;
}

void next_result_block(tlim_ctx* c) {
    c->res_cur ^= 1;
    c->res_host = c->res_blk[c->res_cur];
    c->res_host_dev = c->res_blk_dev[c->res_cur];
}

// Steps that may run pipelined: predicted schedule, no report, no viscous
// part, no total energy, no timing, equal p_inf, 2D without sources (fused relaxation, whose
// relaxed alpha2 and T^n go to fresh arrays).
// A pipelined step is predicted from the step two back, and a miss costs the
// newer step too, so pipelining waits until two consecutive steps kept the
// same schedule.
bool pipeline_ok(const tlim_ctx* c, const tlim_step_opts* o, const tlim_step_report* rep) {
    return !rep && !o->do_viscous && !o->time_sweeps && !o->cycle_mode && !o->frozen_lambda && o->picard_tol <= 0.0 &&
           !c->fset[TLIM_E] &&
           c->phase[0].pinf == c->phase[1].pinf && fast_coeffs(c, dev_grid(c, kUnit)) &&
           c->hist_passes == o->passes && c->hist_steady >= 2 && c->res_host_dev != nullptr;
}

// Enqueue a predicted step without waiting for anything: relaxation with the
// first coefficients, the passes with the predicted P, and the fold of the
// step's reductions into its own pinned result block, which ends with the
// step's sequence number.
void enqueue_predicted(tlim_ctx* c, const tlim_step_opts* o, tlim_ctx::Pending& p) {
    hipStream_t s = c->stream;
    DevGrid g = dev_grid(c, kUnit);
    DevPhases ph = dev_phases(c);
    next_result_block(c);
    relax_step(c, o);
    Timer tm{c, false};
    SweepCount sc;
    bool coef_ready = true;  // the first pass's coefficients come with the relaxation
    for (int it = 0; it < o->passes; ++it) {
        if (!coef_ready) heat_coeffs(c, g, ph, o, row(c, tlim::tgt_lam(it)), it);
        const double* Tit = it == 0 ? c->Tn : c->field[TLIM_T1];
        const int P = c->hist_P[it];
        p.P_used[it] = P;
        PassSchedule ps = device_schedule(P, o->order, row(c, tlim::tgt_lam(it)));
        const bool last = it + 1 == o->passes;
        const bool want = !last && next_coef_ok(c, g);
        const bool want_step = last && next_step_ok(c, o, g);
        tlim::NextCoef nc = want_step ? next_step_coef(c, o, ph) : next_coef(c, it, ph);
        bool done = false;
        // (a pipelined step has neither a report nor a Picard tolerance)
        run_lim_pass(c, g, o->face_mean, o->dt, ps, c->Tn, c->g_heat, c->Tnew, Tit, pass_slots(c, it, false), tm, sc,
                     true, nullptr, want || want_step ? &nc : nullptr, &done);
        coef_ready = false;
        if (want_step) note_next_step(c, o, done);
        else if (done) {
            coef_ready = true;
            adopt_next_coef(c);
        }
        std::swap(c->field[TLIM_T1], c->Tnew);
    }
    const bool move = c->next_ready;
    // the step's results and then its sequence number go to its pinned
    // block: the host polls that number (an event between steps costs about
    // 5 us of idle GPU)
    const unsigned long long seq = ++c->res_seq;
    tlim::launch_collect(s, c->acc, c->res_host_dev, tlim::tgt_lam(0), tlim::tgt_lam(o->passes), 1,
                         move ? tlim::kTgtNextStep : -1, seq, c->collect_done);
    c->clean_rows = c->clean_keep;
    if (move) {
        c->row0_moved = true;
        c->spare_clean = true;
    }
    p.seq = seq;
    p.o = *o;
    p.o.frozen_lambda = nullptr;
    p.o.frozen_visc = nullptr;
    p.blk = c->res_cur;
    p.Tn = c->Tn;
    p.alpha2 = c->field[TLIM_ALPHA2];
    p.alpha2_other = c->a2n;
    p.whole = false;
}

// Steps the whole-step kernel may run pipelined (its P needs no prediction):
// no report, no viscous part, no total energy, no timing.
bool pipeline_whole_ok(const tlim_ctx* c, const tlim_step_opts* o, const tlim_step_report* rep) {
    return o->whole_step == TLIM_WHOLE_ALWAYS && !rep && !o->do_viscous && !o->time_sweeps && !c->fset[TLIM_E] &&
           c->res_host_dev != nullptr && step2d_ok(c, o);
}

// Enqueue a whole-step kernel step and the fold of its rows into its own
// pinned block, followed by an event.  False: the launch was refused.
bool enqueue_whole(tlim_ctx* c, const tlim_step_opts* o, tlim_ctx::Pending& p) {
    next_result_block(c);
    if (!step2d_enqueue(c, o, c->res_host_dev)) return false;
    (void)hipEventRecord(c->ev_pend[c->res_cur], c->stream);
    p.seq = 0;
    p.o = *o;
    p.o.frozen_lambda = nullptr;
    p.o.frozen_visc = nullptr;
    p.blk = c->res_cur;
    p.Tn = c->Tn;
    p.alpha2 = c->field[TLIM_ALPHA2];
    p.alpha2_other = c->a2n;
    p.whole = true;
    return true;
}

struct Verdict {
    tlim_status st;
    bool mispredicted;
    double bad;
    double lam[TLIM_MAX_PASSES];  // the step's lambda_G per pass
};

// Wait for a pending step's readback (polled, like read_result) and check
// the P it used in every pass against its lambda_G.
Verdict verify(tlim_ctx* c, const tlim_ctx::Pending& p) {
    Verdict v{TLIM_OK, false, 0.0, {0}};
    PassResult* res = c->res_blk[p.blk];
    hipError_t r = hipErrorNotReady;
    if (p.seq) {
        bool seen = false;
        r = wait_fold(c, res, p.seq, &seen);
        if (r == hipSuccess && !seen) {
            v.st = fail(c, TLIM_E_HIP, "pipelined step: the stream drained without the step's results");
            return v;
        }
    } else {
        hipEvent_t e = c->ev_pend[p.blk];
        const auto t0c = std::chrono::steady_clock::now();
        while ((r = hipEventQuery(e)) == hipErrorNotReady) {
            if (std::chrono::steady_clock::now() - t0c > std::chrono::microseconds(2000)) {
                r = hipEventSynchronize(e);
                break;
            }
        }
    }
    if (r != hipSuccess) {
        v.st = fail(c, TLIM_E_HIP, "pipelined step: %s", hipGetErrorString(r));
        return v;
    }
    const int np = p.o.passes;
    if (p.whole) {
        Step2DResult r;
        step2d_result(res, np, r);
        if (r.timeout) {
            v.st = lose_heat_state(c);
            return v;
        }
        v.mispredicted = r.out_of_range;  // redone with one launch per block of stages
        for (int i = 0; i < np; ++i) v.lam[i] = r.lam[i];
    } else {
        for (int i = 0; i < np; ++i) {
            v.lam[i] = res->v[tlim::tgt_lam(i)];
            if (lim_P(p.o.dt, v.lam[i]) != p.P_used[i]) v.mispredicted = true;
        }
    }
    v.bad = res->v[tlim::tgt_bad(np - 1)];
    return v;
}

// Redo the passes of a mispredicted step from its relaxed state, with one
// readback per pass.
tlim_status redo_pending(tlim_ctx* c, const tlim_ctx::Pending& p) {
    c->Tn = p.Tn;
    c->g_heat = p.Tn;
    c->field[TLIM_ALPHA2] = p.alpha2;
    c->a2n = p.alpha2_other;
    for (double* a : c->a2pool)  // a2x: the third alpha2 array
        if (a != c->field[TLIM_ALPHA2] && a != c->a2n) c->a2x = a;
    c->predict_misses++;
    c->pipeline_redos++;
    Timer tm{c, false};
    SweepCount sc;
    HeatOutcome out;
    tlim_status st = heat_passes(c, &p.o, Mode::Sync, nullptr, tm, sc, out, false);
    if (st) return st;
    if (out.bad > 0.0) return fail(c, TLIM_E_NUMERIC, "%.0f cells with non-finite or non-positive T", out.bad);
    return TLIM_OK;
}

// Verify the pending step, if any (redoing it when mispredicted); every entry
// point that reads or changes the state calls this first.
tlim_status resolve(tlim_ctx* c) {
    if (!c || !c->pending) return TLIM_OK;
    c->pending = false;
    const tlim_ctx::Pending p = c->pend;
    Verdict v = verify(c, p);
    if (v.st) return v.st;
    if (v.mispredicted) return redo_pending(c, p);
    record_schedule(c, p.o.passes, v.lam, p.o.dt);
    if (v.bad > 0.0) return fail(c, TLIM_E_NUMERIC, "%.0f cells with non-finite or non-positive T", v.bad);
    return TLIM_OK;
}

}  // namespace

tlim_status tlim_advance_parabolic(tlim_ctx* c, const tlim_step_opts* o, tlim_step_report* rep) {
    if (!c) return TLIM_E_ARG;
    tlim_status st = check_opts(c, o);
    if (st) return st;
    st = check_ready(c);
    if (st) return st;
    const bool whole = pipeline_whole_ok(c, o, rep) && step2d_table(c, o->order) == TLIM_OK;
    if (!whole && !pipeline_ok(c, o, rep)) {
        st = resolve(c);
        if (st) return st;
        return advance_sync(c, o, rep);
    }
    // Pipelined: enqueue this step first, then verify the previous one while
    // this one runs.
    tlim_ctx::Pending np{};
    if (whole) {
        if (!enqueue_whole(c, o, np)) {
            st = resolve(c);
            if (st) return st;
            return advance_sync(c, o, rep);
        }
    } else {
        enqueue_predicted(c, o, np);
    }
    c->pipelined_steps++;
    if (!c->pending) {
        c->pending = true;
        c->pend = np;
        return TLIM_OK;
    }
    const tlim_ctx::Pending prev = c->pend;
    c->pending = false;
    Verdict v = verify(c, prev);
    if (v.st) return v.st;
    if (v.mispredicted) {
        // this step started from a state that is redone: let it finish,
        // redo the previous step, then run this one with its own readback
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        st = redo_pending(c, prev);
        if (st) return st;
        return advance_sync(c, o, nullptr);
    }
    record_schedule(c, prev.o.passes, v.lam, prev.o.dt);
    c->pending = true;
    c->pend = np;
    if (v.bad > 0.0)
        return fail(c, TLIM_E_NUMERIC, "%.0f cells with non-finite or non-positive T (previous step)", v.bad);
    return TLIM_OK;
}

tlim_status tlim_finish(tlim_ctx* c) {
    if (!c) return TLIM_E_ARG;
    return resolve(c);
}

// ------------------------------------------------------------------ adjoint

namespace {

tlim_status check_adjoint(tlim_ctx* c, const tlim_step_opts* o) {
    c->next_ready = false;  // the adjoint runs its own steps on the fields
    tlim_status st = check_opts(c, o);
    if (st) return st;
    st = check_ready(c);
    if (st) return st;
    if (c->phase[0].pinf != c->phase[1].pinf) return fail(c, TLIM_E_ARG, "adjoint needs equal p_inf of both phases");
    if (o->cycle_mode || o->do_viscous || o->picard_tol > 0.0)
        return fail(c, TLIM_E_ARG, "adjoint runs plain LIM heat steps (no cycle mode, viscous part or Picard tol)");
    if (c->fset[TLIM_SRC1] || c->fset[TLIM_SRC2]) return fail(c, TLIM_E_ARG, "adjoint runs without heat sources");
    if (c->fset[TLIM_E]) return fail(c, TLIM_E_ARG, "adjoint runs without the total energy field");
    return TLIM_OK;
}

// Adjoint workspace: `keep` step blocks (every stage of every pass, the pass
// iterates and the conductivities of one recomputed step; block k at
// k * step), then the adjoint fields shared by all steps.
struct AdjLayout {
    size_t stages, Tpass, Lp, step, mu, acc, dg, gLam, lamA, lamB, total;
    int nst, keep;
};

AdjLayout adj_layout(int64_t N, int passes, int Pmax, int keep = 1) {
    AdjLayout L{};
    size_t d = align_up(sizeof(double) * (size_t)N);
    L.nst = 2 * Pmax - 1;
    L.keep = keep;
    size_t off = 0;
    L.stages = off;
    off += d * (size_t)passes * (size_t)L.nst;
    L.Tpass = off;
    off += d * (size_t)(passes + 1);
    L.Lp = off;
    off += d * (size_t)passes;
    L.step = off;
    off = L.step * (size_t)keep;
    size_t* rest[] = {&L.mu, &L.acc, &L.dg, &L.gLam, &L.lamA, &L.lamB};
    for (size_t* p : rest) {
        *p = off;
        off += d;
    }
    L.total = off;
    return L;
}

// Heat passes of one step without relaxation, from T0: pass it reads
// T^(it) (T0 for it = 0, else Tpass + it*sf) and writes T^(it+1) to
// Tpass + (it+1)*sf.  With stages != NULL every stage iterate v^(m),
// 1 <= m < nst, of pass it goes to slot m of stages + it*stride_pass
// (v^(0) = T0 is not copied), and the conductivities of pass it to
// Lp + it*sf.  1/C is built by the first pass that finds rC_ready false.
void adj_forward_step(tlim_ctx* c, const tlim_step_opts* o, const double* lamv, const double* T0, double* Tpass,
                      double* stages, double* Lp, size_t sf, size_t stride_pass, bool& rC_ready) {
    DevGrid g = dev_grid(c, kUnit);
    DevPhases ph = dev_phases(c);
    hipStream_t s = c->stream;
    for (int it = 0; it < o->passes; ++it) {
        const double* Tit = it == 0 ? T0 : Tpass + (size_t)it * sf;
        double* Tout = Tpass + (size_t)(it + 1) * sf;
        double* Lam = Lp ? Lp + (size_t)it * sf : c->Lam;
        // no sources: g = T0, and no right-hand side is written
        tlim::launch_heat_coeffs(s, g, ph, o->alpha_eps, o->dt, Tit, c->field[TLIM_ALPHA2], c->field[TLIM_M1],
                                 c->field[TLIM_M2], T0, nullptr, nullptr, Lam, rC_ready ? nullptr : c->rC, nullptr,
                                 nullptr, nullptr);
        rC_ready = true;
        int P = lim_P(o->dt, lamv[it]);
        std::vector<double> b = lim_params(P, lamv[it], o->order);
        int nst = (int)b.size();
        std::vector<double> tbv(nst);
        for (int m = 0; m < nst; ++m) tbv[m] = o->dt * b[m];
        if (stages) {
            double* st0 = stages + (size_t)it * stride_pass;
            auto vin = [&](int m) -> const double* { return m == 0 ? T0 : st0 + (size_t)m * sf; };
            int m = 0;
            while (m < nst) {
                int k = tlim::sweeps_per_launch(g, nst - m);
                double* out = m + k == nst ? Tout : st0 + (size_t)(m + k) * sf;
                tlim::Stages stg{nullptr, tbv.data() + m, nullptr};
                int done = -1;
                if (k > 1)
                    done = tlim::launch_sweeps64_keep(s, g, o->face_mean, vin(m), T0, Lam, c->rC, out, stg, k, o->dt,
                                                      st0 + (size_t)m * sf, (int64_t)sf);
                if (done < 0) {
                    // one stage into its own slot, by the kernel the forward
                    // run uses for this grid (z-marching waves in 3D)
                    double* one = m + 1 == nst ? Tout : st0 + (size_t)(m + 1) * sf;
                    tlim::Stages s1{nullptr, tbv.data() + m, nullptr};
                    done = tlim::launch_sweeps64(s, g, o->face_mean, vin(m), T0, Lam, c->rC, one, s1, 1, m + 1 == nst,
                                                 o->dt, nullptr, tlim::PassSlots{});
                }
                m += done;
            }
        } else {
            const double* cur = T0;
            int pp = 0, m = 0;
            while (m < nst) {
                int k = tlim::sweeps_per_launch(g, nst - m);
                bool last = m + k == nst;
                double* nxt = last ? Tout : c->vb[pp];
                tlim::Stages stg{nullptr, tbv.data() + m, nullptr};
                m += tlim::launch_sweeps64(s, g, o->face_mean, cur, T0, Lam, c->rC, nxt, stg, k, last, o->dt, nullptr,
                                           tlim::PassSlots{});
                cur = nxt;
                pp ^= 1;
            }
        }
    }
}

}  // namespace

tlim_status tlim_forward_checkpointed(tlim_ctx* c, const tlim_step_opts* o, int32_t nsteps, int32_t ckpt_every,
                                      double* ckpt_dev, double* lam_out) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    tlim_status st = check_adjoint(c, o);
    if (st) return st;
    if (nsteps < 1 || ckpt_every < 1 || !ckpt_dev || !lam_out) return fail(c, TLIM_E_ARG, "bad checkpoint arguments");
    if (o->frozen_lambda) return fail(c, TLIM_E_ARG, "the forward run records its own schedule");
    for (int n = 0; n < nsteps; ++n) {
        if (n % ckpt_every == 0)
            tlim::launch_copy(c->stream, ckpt_dev + (size_t)(n / ckpt_every) * (size_t)c->N, c->field[TLIM_T1], c->N);
        tlim_step_report rep;
        st = tlim_advance_parabolic(c, o, &rep);
        if (st) return st;
        for (int it = 0; it < o->passes; ++it) lam_out[(size_t)n * o->passes + it] = rep.lambda_G[it];
    }
    return TLIM_OK;
}

tlim_status tlim_adjoint_workspace_bytes(const tlim_ctx* c, const tlim_step_opts* o, int32_t nsteps,
                                         const double* lam, size_t* bytes) {
    if (!c || !o || !bytes || !lam || nsteps < 1 || o->passes < 1 || o->passes > TLIM_MAX_PASSES ||
        !(o->dt > 0.0) || !std::isfinite(o->dt))
        return TLIM_E_ARG;
    int Pmax = 1;
    for (int k = 0; k < nsteps * o->passes; ++k) {
        if (!(lam[k] >= 0.0) || !std::isfinite(lam[k])) return TLIM_E_ARG;
        Pmax = std::max(Pmax, lim_P(o->dt, lam[k]));
    }
    *bytes = adj_layout(c->N, o->passes, Pmax).total;
    return TLIM_OK;
}

tlim_status tlim_adjoint_workspace_bytes_kept(const tlim_ctx* c, const tlim_step_opts* o, int32_t nsteps,
                                              int32_t ckpt_every, const double* lam, size_t* bytes) {
    if (ckpt_every < 1) return TLIM_E_ARG;
    tlim_status st = tlim_adjoint_workspace_bytes(c, o, nsteps, lam, bytes);
    if (st) return st;
    int Pmax = 1;
    for (int k = 0; k < nsteps * o->passes; ++k) Pmax = std::max(Pmax, lim_P(o->dt, lam[k]));
    *bytes = adj_layout(c->N, o->passes, Pmax, std::min(ckpt_every, nsteps)).total;
    return TLIM_OK;
}

tlim_status tlim_adjoint_parabolic(tlim_ctx* c, const tlim_step_opts* o, int32_t nsteps, int32_t ckpt_every,
                         const double* ckpt_dev, const double* lam, const double* dL_dTN_dev, double* dL_dT0_dev,
                         double* dL_dk0, void* adj_ws_dev, size_t adj_ws_bytes) {
    if (!c) return TLIM_E_ARG;
    tlim_status pst = resolve(c);
    if (pst) return pst;
    tlim_status st = check_adjoint(c, o);
    if (st) return st;
    if (nsteps < 1 || ckpt_every < 1 || !ckpt_dev || !lam || !dL_dTN_dev || !dL_dT0_dev || !dL_dk0 || !adj_ws_dev)
        return fail(c, TLIM_E_ARG, "bad adjoint arguments");
    if (((uintptr_t)adj_ws_dev % kAlign) != 0) return fail(c, TLIM_E_ARG, "adjoint workspace not 256-byte aligned");
    const int np = o->passes;
    int Pmax = 1;
    for (int k = 0; k < nsteps * np; ++k) {
        if (!(lam[k] >= 0.0) || !std::isfinite(lam[k])) return fail(c, TLIM_E_ARG, "schedule entry %d invalid", k);
        Pmax = std::max(Pmax, lim_P(o->dt, lam[k]));
    }
    AdjLayout L = adj_layout(c->N, np, Pmax);
    if (adj_ws_bytes < L.total) return fail(c, TLIM_E_NOMEM, "adjoint workspace %zu < %zu bytes", adj_ws_bytes, L.total);
    // A workspace with a block for every step of a checkpoint interval keeps
    // them all: the interval is recomputed once, when its last step comes
    // up, instead of its first steps once more for each later step.
    const int keep = std::min(ckpt_every, nsteps);
    if (keep > 1) {
        const AdjLayout Lk = adj_layout(c->N, np, Pmax, keep);
        if (adj_ws_bytes >= Lk.total) L = Lk;
    }
    char* base = (char*)adj_ws_dev;
    const size_t sf = align_up(sizeof(double) * (size_t)c->N) / sizeof(double);  // doubles per field slot
    auto block = [&](int k, size_t off) { return (double*)(base + (size_t)k * L.step + off); };
    double* stages = block(0, L.stages);
    double* Tpass = block(0, L.Tpass);
    double* mu = (double*)(base + L.mu);
    double* acc = (double*)(base + L.acc);
    double* dg = (double*)(base + L.dg);
    double* gLam = (double*)(base + L.gLam);
    double* lamA = (double*)(base + L.lamA);
    double* lamB = (double*)(base + L.lamB);
    const size_t stride_pass = sf * (size_t)L.nst;
    hipStream_t s = c->stream;
    DevGrid g = dev_grid(c, kUnit);
    DevPhases ph = dev_phases(c);
    const int64_t N = c->N;
    double k0g[2] = {0.0, 0.0};

    double* Lp = block(0, L.Lp);
    bool rC_ready = false;
    tlim::launch_copy(s, mu, dL_dTN_dev, N);
    // dL/dk0 sums accumulate on the device over all passes and steps
    zero_rows(c, tlim::kTgtK0a, tlim::kTgtK0b + 1);
    for (int n = nsteps - 1; n >= 0; --n) {
        // T^n from the nearest checkpoint at or before n
        const int base_step = (n / ckpt_every) * ckpt_every;
        const double* T0 = ckpt_dev + (size_t)(n / ckpt_every) * (size_t)N;
        if (L.keep > 1) {
            // every step of the interval recomputed once, each into its own
            // block (keeping every stage and every pass's conductivities),
            // when the interval's last step comes up
            const int blk = n - base_step;
            if (n == std::min(nsteps, base_step + ckpt_every) - 1) {
                const double* t = T0;
                for (int m = base_step; m <= n; ++m) {
                    const int k = m - base_step;
                    adj_forward_step(c, o, lam + (size_t)m * np, t, block(k, L.Tpass), block(k, L.stages),
                                     block(k, L.Lp), sf, stride_pass, rC_ready);
                    t = block(k, L.Tpass) + (size_t)np * sf;
                }
            }
            if (blk > 0) T0 = block(blk - 1, L.Tpass) + (size_t)np * sf;
            stages = block(blk, L.stages);
            Tpass = block(blk, L.Tpass);
            Lp = block(blk, L.Lp);
        } else {
            for (int m = base_step; m < n; ++m) {
                adj_forward_step(c, o, lam + (size_t)m * np, T0, Tpass, nullptr, nullptr, sf, stride_pass, rC_ready);
                tlim::launch_copy(s, Tpass, Tpass + (size_t)np * sf, N);
                T0 = Tpass;
            }
            // recompute step n keeping every stage and every pass's conductivities
            adj_forward_step(c, o, lam + (size_t)n * np, T0, Tpass, stages, Lp, sf, stride_pass, rC_ready);
        }
        for (int it = np - 1; it >= 0; --it) {
            const double* Tit = it == 0 ? T0 : Tpass + (size_t)it * sf;
            const double* Lam = Lp + (size_t)it * sf;
            int P = lim_P(o->dt, lam[(size_t)n * np + it]);
            std::vector<double> b = lim_params(P, lam[(size_t)n * np + it], o->order);
            int nst = (int)b.size();
            const double* cur = mu;
            double* bufs[2] = {lamA, lamB};
            int pp = 0;
            const double* st0 = stages + (size_t)it * stride_pass;
            // blocked reverse stages in psi = C^-1 lambda form where the grid
            // allows; the launch that reaches v^(0) also finishes the pass
            bool psi_form = false, cell_done = false;
            tlim::AdjCell cell{ph, Tit, c->field[TLIM_ALPHA2], c->field[TLIM_M1], c->field[TLIM_M2], acc, mu,
                               it == np - 1 ? 1 : 0, it == 0 ? 1 : 0,
                               row(c, tlim::kTgtK0a), row(c, tlim::kTgtK0b)};
            {
                std::vector<double> cmv, tbv;
                int m = nst;
                while (m >= 1) {
                    int k = std::min(m, tlim::sweeps_per_launch(g, m));
                    cmv.assign(k, 0.0);
                    tbv.assign(k, 0.0);
                    for (int q = 0; q < k; ++q) {
                        tbv[q] = o->dt * b[m - 1 - q];
                        cmv[q] = 1.0 / (1.0 + tbv[q]);
                    }
                    int done = tlim::launch_adjoint_sweeps(s, g, o->face_mean, cur, m == nst ? 1 : 0, Lam, c->rC, st0,
                                                           T0, (int64_t)sf, m, bufs[pp], dg, gLam, m == nst ? 0 : 1,
                                                           cmv.data(), tbv.data(), k, o->dt, &cell);
                    if (done < 0) break;
                    psi_form = true;
                    if (m - done == 0) cell_done = true;
                    cur = bufs[pp];
                    pp ^= 1;
                    m -= done;
                }
            }
            if (!psi_form && tlim::use_adj_z3d(g, o->face_mean)) {
                // 3D grids: reverse stages by z-marching waves in psi form
                tlim::launch_fill(s, dg, 0.0, N);
                tlim::launch_fill(s, gLam, 0.0, N);
                tlim::launch_psi_from_lambda(s, N, cur, c->rC, bufs[pp]);
                cur = bufs[pp];
                pp ^= 1;
                for (int m = nst; m >= 1; --m) {
                    const double tb = o->dt * b[m - 1];
                    const double* vprev = m == 1 ? T0 : st0 + (size_t)(m - 1) * sf;
                    tlim::launch_adj_z3d(s, g, cur, vprev, Lam, c->rC, bufs[pp], dg, gLam, 1.0 / (1.0 + tb), tb,
                                         o->dt);
                    cur = bufs[pp];
                    pp ^= 1;
                }
                psi_form = true;
            }
            if (!psi_form) {
                tlim::launch_fill(s, dg, 0.0, N);
                tlim::launch_fill(s, gLam, 0.0, N);
                for (int m = nst; m >= 1; --m) {
                    double tb = o->dt * b[m - 1];
                    const double* vprev = m == 1 ? T0 : st0 + (size_t)(m - 1) * sf;
                    tlim::launch_adj_stage(s, g, o->face_mean, cur, vprev, Lam, c->rC, bufs[pp], dg, gLam,
                                           1.0 / (1.0 + tb), tb, o->dt);
                    cur = bufs[pp];
                    pp ^= 1;
                }
            }
            // cur = dL/dv^(0) (or its psi); mu <- dL/dT^(it) through Lambda(T^(it));
            // the last pass (reversed first) starts the step's sum acc
            if (!cell_done)
                tlim::launch_adj_cell(s, g, ph, Tit, c->field[TLIM_ALPHA2], c->field[TLIM_M1], c->field[TLIM_M2],
                                      gLam, dg, cur, acc, mu, it == 0 ? 1 : 0,
                                      psi_form ? c->rC : nullptr, row(c, tlim::kTgtK0a), row(c, tlim::kTgtK0b),
                                      it == np - 1 ? 1 : 0);
        }
        std::swap(mu, acc);  // dL/dT^n seeds step n-1
    }
    st = read_result(c, tlim::kTgtK0a, tlim::kTgtK0b + 1);
    if (st) return st;
    k0g[0] = result(c, tlim::kTgtK0a);
    k0g[1] = result(c, tlim::kTgtK0b);
    tlim::launch_copy(s, dL_dT0_dev, mu, N);
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipGetLastError());
    dL_dk0[0] = k0g[0];
    dL_dk0[1] = k0g[1];
    return TLIM_OK;
}

}  // extern "C"
