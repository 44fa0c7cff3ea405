/*
 * Host sanitizer run of the library's argument checks and checkpoint parser:
 * linked against a libns whose host code is built under AddressSanitizer and
 * UndefinedBehaviorSanitizer, it calls the entry points with invalid
 * arguments and ns_load with malformed checkpoints (wrong magic, truncated,
 * random bytes after a valid magic, huge array counts).  Every call must be
 * refused with NS_E_ARG before anything reaches a GPU, so the program runs
 * on a host without one.  Exit status 0 when every call is refused as
 * expected; the sanitizers abort on the first memory or undefined-behaviour
 * error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ns.h"

static int fails = 0;

static void expect(int rc, int want, const char* what) {
    const char* msg = ns_last_error();
    if (rc != want || msg == NULL) {
        fprintf(stderr, "%s: returned %d, expected %d (%s)\n", what, rc, want, msg ? msg : "no message");
        ++fails;
    }
}

int main(void) {
    int kind[2] = {NS_PRIOR_UNIFORM, NS_PRIOR_UNIFORM};
    double lo[2] = {0, 0}, hi[2] = {1, 1}, mu[2] = {0.5, 0.5};
    ns_problem p;
    memset(&p, 0, sizeof p);
    p.likelihood = NS_LIKE_GAUSS;
    p.n_dim = 2;
    p.prior_kind = kind; p.prior_lo = lo; p.prior_hi = hi;
    p.f_lo = 1.0; p.df = 1.0;
    p.gauss_mu = mu; p.gauss_sigma = 0.1;
    ns_opts o;
    memset(&o, 0, sizeof o);
    o.n_live = 100; o.n_delete = 50; o.n_steps = 10; o.slice_width = 1.0;
    o.max_stepout = 10; o.max_shrink = 10; o.term_frac = 1e-3; o.max_iter = 10;
    o.precision = NS_FP64; o.kernel = NS_KERNEL_SLICE; o.walk_accept = 1; o.walk_max = 1;

    ns_run* run = NULL;
    expect(ns_init(NULL, &p, &o, NULL), NS_E_ARG, "ns_init without out");
    expect(ns_init(&run, NULL, &o, NULL), NS_E_ARG, "ns_init without problem");
    expect(ns_init(&run, &p, NULL, NULL), NS_E_ARG, "ns_init without opts");
    ns_problem q = p;
    q.n_dim = 0;
    expect(ns_init(&run, &q, &o, NULL), NS_E_ARG, "n_dim 0");
    q = p;
    q.n_dim = 13;
    expect(ns_init(&run, &q, &o, NULL), NS_E_ARG, "n_dim 13");
    q = p;
    q.gauss_sigma = 0.0;
    expect(ns_init(&run, &q, &o, NULL), NS_E_ARG, "gauss_sigma 0");
    q = p;
    q.likelihood = 7;
    expect(ns_init(&run, &q, &o, NULL), NS_E_ARG, "likelihood 7");
    const struct { const char* what; ns_opts o; } bad[] = {
        {"n_live 1", {.n_live = 1}}, {"n_delete = n_live", {.n_live = 100, .n_delete = 100}},
    };
    for (size_t i = 0; i < sizeof bad / sizeof bad[0]; ++i) expect(ns_init(&run, &p, &bad[i].o, NULL), NS_E_ARG, bad[i].what);
    ns_opts b = o;
    b.n_steps = 0; expect(ns_init(&run, &p, &b, NULL), NS_E_ARG, "n_steps 0");
    b = o; b.slice_width = 0.0; expect(ns_init(&run, &p, &b, NULL), NS_E_ARG, "slice_width 0");
    b = o; b.max_iter = 0; expect(ns_init(&run, &p, &b, NULL), NS_E_ARG, "max_iter 0");
    b = o; b.precision = 2; expect(ns_init(&run, &p, &b, NULL), NS_E_ARG, "precision 2");
    b = o; b.kernel = 2; expect(ns_init(&run, &p, &b, NULL), NS_E_ARG, "kernel 2");
    b = o; b.count_moves = 2; expect(ns_init(&run, &p, &b, NULL), NS_E_ARG, "count_moves 2");
    if (run != NULL) { fprintf(stderr, "a refused ns_init left a run\n"); ++fails; }

    expect(ns_select(NULL, 10, 5, NULL, NULL, NULL), NS_E_ARG, "ns_select without arrays");
    expect(ns_step(NULL, 1, NULL), NS_E_ARG, "ns_step without run");
    expect(ns_trace(NULL, 0, NULL, NULL), NS_E_ARG, "ns_trace without run");

    /* checkpoints */
    expect(ns_load(NULL, "x", 1, NULL), NS_E_ARG, "ns_load without out");
    expect(ns_load(&run, NULL, 8, NULL), NS_E_ARG, "ns_load without buffer");
    expect(ns_load(&run, "NSRUNv1", 8, NULL), NS_E_ARG, "old checkpoint magic");
    expect(ns_load(&run, "NSRU", 4, NULL), NS_E_ARG, "short buffer");
    unsigned char buf[4096];
    memcpy(buf, "NSRUNv3", 8);
    uint64_t s = 0x9e3779b97f4a7c15ull;
    for (int trial = 0; trial < 3000; ++trial) {
        const size_t size = 8 + (size_t)(trial * 37 % 4000);
        for (size_t i = 8; i < size; ++i) {
            s ^= s << 13; s ^= s >> 7; s ^= s << 17;    /* xorshift64 */
            buf[i] = (unsigned char)(s >> 24);
        }
        if (trial % 3 == 0 && size >= 8 + 4 + 8) {
            /* a plausible header, then a huge array count */
            memset(buf + 8, 0, 4);
            uint64_t huge = (uint64_t)1 << 62;
            memcpy(buf + size - 8, &huge, 8);
        }
        run = NULL;
        const int rc = ns_load(&run, buf, size, NULL);
        if (rc != NS_E_ARG || run != NULL) {
            fprintf(stderr, "malformed checkpoint %d (size %zu) returned %d\n", trial, size, rc);
            ++fails;
            break;
        }
    }
    printf("ns_host_sanitize: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
