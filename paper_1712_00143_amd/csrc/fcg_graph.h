// Captured iteration chunks of the sloppy solver loops, and the choice of how
// many iterations to run before the host next reads the solver state.
//
// The device pauses a loop (status no longer running) when |r|^2 falls below
// max(tol^2 |b|^2, delta^2 max|r|^2): a reliable update or the convergence
// check is due.  Launches already queued behind that point are status-gated
// and exit at once, but each still costs a dispatch, so a fixed chunk of k
// iterations wastes about k/2 gated iterations per pause.  Once the
// residual's decay rate is known, ChunkPlanner sizes the next chunk to end
// where |r|^2 is expected to cross the threshold; ChunkGraphs holds captured
// chunks of k and of every power of two below k, so that any length is a few
// back-to-back graph launches.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "hisq_dev.h"

namespace hisq {

struct ChunkGraphs {
    static constexpr int MAXG = 12;
    int n = 0;
    int len[MAXG] = {};   // iterations per graph, decreasing
    hipGraph_t graph[MAXG] = {};
    hipGraphExec_t exec[MAXG] = {};
    std::string key;      // every launch argument the chunks hold by value
    void release()
    {
        for (int i = 0; i < n; i++) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
            exec[i] = nullptr;
            graph[i] = nullptr;
        }
        n = 0;
        key.clear();
    }
    bool ready() const { return n > 0; }
    // lengths k, then the powers of two below k (the smallest MAXG - 1 of
    // them, so that 1 is always there and every count can be launched)
    static int lengths(int k, int out[MAXG])
    {
        int pw[MAXG], np = 0;
        for (int p = 1; p < k && np < MAXG - 1; p *= 2) pw[np++] = p;
        int m = 0;
        out[m++] = k;
        while (np > 0) out[m++] = pw[--np];
        return m;
    }
    // capture every length: enqueue(len) puts len iterations on s
    template <class F>
    hipError_t capture(int k, hipStream_t s, F &&enqueue)
    {
        release();
        int ls[MAXG];
        const int m = lengths(k, ls);
        for (int i = 0; i < m; i++) {
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            hipError_t ce = enqueue(ls[i]);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(s, &g);
            if (ce != hipSuccess || ee != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return ce != hipSuccess ? ce : ee;
            }
            len[n] = ls[i];
            graph[n] = g;
            exec[n] = nullptr;
            n++;
            e = hipGraphInstantiate(&exec[n - 1], g, nullptr, nullptr, 0);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // iters iterations as graph launches, largest lengths first (the last
    // length is 1, so every count is reached)
    hipError_t launch(int iters, hipStream_t s) const
    {
        for (int i = 0; i < n && iters > 0;) {
            if (len[i] <= iters) {
                hipError_t e = hipGraphLaunch(exec[i], s);
                if (e != hipSuccess) return e;
                iters -= len[i];
            } else {
                i++;
            }
        }
        return iters > 0 ? hipErrorInvalidValue : hipSuccess;
    }
};

// Decay rate of |r|^2 per iteration, observed at the host's reads of a
// running solve, and the chunk length it suggests.
struct ChunkPlanner {
    int kmax = 16;
    double rate = 0.0;   // mean d ln|r|^2 / d iteration (< 0 once known)
    int last_iter = -1;
    double last_rr = 0.0;
    explicit ChunkPlanner(int k) : kmax(k) {}
    // the state at a host read after a chunk, running or paused (the paused
    // state still holds the recursion's |r|^2 and iteration count)
    void observe(const SolveState &st)
    {
        if (last_iter >= 0 && st.iter > last_iter && st.rr > 0.0 && last_rr > 0.0) {
            const double g = std::log(st.rr / last_rr) / (double)(st.iter - last_iter);
            if (g < 0.0) rate = rate < 0.0 ? 0.5 * (rate + g) : g;
        }
        rebase(st);
    }
    // the recursion starts again from st.rr (start, or after a reliable update)
    void rebase(const SolveState &st)
    {
        last_iter = st.iter;
        last_rr = st.rr;
    }
    // iterations until |r|^2 is expected below the pause threshold, in [1, kmax]
    int next(const SolveState &st) const
    {
        int n = kmax;
        if (rate < 0.0 && st.rr > 0.0) {
            const double thr = std::max(st.tol2 * st.bb, st.delta2 * st.maxrr);
            const double need = st.rr > thr ? std::log(thr / st.rr) / rate : 1.0;
            if (need < (double)kmax) n = std::max(1, (int)std::ceil(need));
        }
        if (st.maxiter > st.iter) n = std::min(n, st.maxiter - st.iter);
        return std::max(1, n);
    }
};

}  // namespace hisq
