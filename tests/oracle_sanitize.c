/*
 * Host sanitizer run of the CPU oracle: this driver is compiled together with oracle/vns_oracle.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py (CPU only) and exercises
 * every exported oracle routine on the instances the test writes to stdin.  It prints, per instance, the
 * results the test compares with the same calls through the unsanitized liboracle.so.
 *
 * Input (whitespace-separated integers), repeated until EOF:
 *   K T seed iters
 *   D[K*T] R[K*T] kM[K] kR[K] hM[K] hR[K] pM[K] pR[K] zM[K*T] zR[K*T]
 * Output per instance, one line each:
 *   obj F                              objective of (zM, zR)
 *   price n_evals sum_of_finite_prices n_finite
 *   vnd F evals n_moves
 *   gvns F F_best k evals sum_of_record_F_local
 *   best_of G literal F F_best k evals
 */
#include <stdio.h>

#include "../oracle/vns_oracle.c"

static int read_i32(int32_t *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (scanf("%d", &a[i]) != 1) return 0;
    return 1;
}

int main(void)
{
    int K, T;
    unsigned long long seed;
    long long iters;
    while (scanf("%d %d %llu %lld", &K, &T, &seed, &iters) == 4) {
        size_t n = (size_t)K * (size_t)T;
        int32_t *D = malloc(sizeof(int32_t) * n), *R = malloc(sizeof(int32_t) * n);
        int32_t *v[6];
        for (int j = 0; j < 6; ++j) v[j] = malloc(sizeof(int32_t) * (size_t)K);
        int32_t *zi = malloc(sizeof(int32_t) * 2 * n);
        if (!read_i32(D, n) || !read_i32(R, n)) return 2;
        for (int j = 0; j < 6; ++j)
            if (!read_i32(v[j], (size_t)K)) return 2;
        if (!read_i32(zi, 2 * n)) return 2;
        uint8_t *zM = malloc(n), *zR = malloc(n), *wM = malloc(n), *wR = malloc(n);
        for (size_t i = 0; i < n; ++i) {
            zM[i] = (uint8_t)zi[i];
            zR[i] = (uint8_t)zi[n + i];
        }
        const int32_t *kM = v[0], *kR = v[1], *hM = v[2], *hR = v[3], *pM = v[4], *pR = v[5];
        int64_t *cost = malloc(sizeof(int64_t) * (size_t)K);
        int64_t F = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, cost);
        printf("obj %lld\n", (long long)F);

        int64_t *price = malloc(sizeof(int64_t) * 4 * n);
        int64_t ev = orc_price_all(K, T, D, R, kM, kR, hM, hR, pM, pR, zM, zR, 7u, price);
        long long sum = 0, nf = 0;
        for (size_t i = 0; i < 4 * n; ++i)
            if (price[i] != ORC_INF) { sum += price[i] % 1000003; ++nf; }
        int64_t slot;
        (void)orc_argmin((int64_t)(4 * n), price, &slot);
        printf("price %lld %lld %lld\n", (long long)ev, sum, nf);

        const int32_t nb[3] = {1, 2, 4};
        memcpy(wM, zM, n);
        memcpy(wR, zR, n);
        int64_t vev = 0, nmoves = 0;
        int64_t *trace = malloc(sizeof(int64_t) * 5 * 64);
        int64_t Fv = orc_vnd_trace(K, T, D, R, kM, kR, hM, hR, pM, pR, wM, wR, nb, 3, &vev, trace, 64, &nmoves);
        printf("vnd %lld %lld %lld\n", (long long)Fv, (long long)vev, (long long)nmoves);

        orc_record *rec = malloc(sizeof(orc_record) * (size_t)(iters > 0 ? iters : 1));
        for (size_t i = 0; i < n; ++i) { wM[i] = 1; wR[i] = 0; }
        int32_t k = 1;
        int64_t Fb = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, wM, wR, NULL), gev = 0;
        int64_t Fg = orc_gvns(K, T, D, R, kM, kR, hM, hR, pM, pR, wM, wR, nb, 3, 5, seed, 0, 0, iters, &k, &Fb,
                              rec, &gev);
        long long sl = 0;
        for (long long i = 0; i < iters; ++i) sl += rec[i].F_local % 1000003;
        printf("gvns %lld %lld %d %lld %lld\n", (long long)Fg, (long long)Fb, k, (long long)gev, sl);

        for (int literal = 0; literal < 2; ++literal) {
            for (size_t i = 0; i < n; ++i) { wM[i] = 1; wR[i] = 0; }
            k = 1;
            Fb = orc_objective(K, T, D, R, kM, kR, hM, hR, pM, pR, wM, wR, NULL);
            int64_t bev = 0;
            int64_t Fo = orc_gvns_best_of(K, T, D, R, kM, kR, hM, hR, pM, pR, wM, wR, nb, 3, 5, 3, literal, seed, 1,
                                          0, iters, &k, &Fb, rec, &bev);
            printf("best_of 3 %d %lld %lld %d %lld\n", literal, (long long)Fo, (long long)Fb, k, (long long)bev);
        }
        free(rec); free(trace); free(price); free(cost);
        free(zM); free(zR); free(wM); free(wR); free(zi);
        for (int j = 0; j < 6; ++j) free(v[j]);
        free(D); free(R);
    }
    return 0;
}
