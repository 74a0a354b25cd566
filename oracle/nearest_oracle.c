/*
 * Plain CPU oracle for exact brute-force nearest-neighbour search.
 *
 * TEST INFRASTRUCTURE ONLY.  Like the correlation oracle beside it, this file
 * is the independent reference that the GPU library is checked against; the
 * library never loads it and shares no code, header or constant with it.
 *
 * The operation is the bottleneck of the natural-image entropy estimate
 * (Sec. 6.4, "Estimating the Entropy of Natural Scenes", and its table of
 * nearest-neighbour search times): for every 8 x 8 target patch (64 pixel
 * values) find, by exhaustive comparison, the patch of a neighbour set at the
 * smallest Euclidean distance.  The answer has to be exact, not approximate.
 * Readings (listed in the design notes): pixels are 8-bit unsigned values,
 * a patch is its D pixel values in a fixed order, the distance reported is
 * the squared Euclidean distance (an integer), and among neighbours at the
 * same smallest distance the one with the lowest index is the answer.
 *
 *   dist[t] = min_m  sum_{d<D} (targets[t][d] - neighbors[m][d])^2
 *   idx[t]  = the smallest m attaining dist[t]
 *
 * Every sum runs sequentially in 64-bit integers in the loop order written;
 * OpenMP only splits the targets between threads.
 */
#include <stdint.h>

typedef int64_t i64;

void nno_search(const uint8_t* targets, const uint8_t* neighbors, i64 T, i64 M, i64 D,
                i64* idx, i64* dist) {
#pragma omp parallel for schedule(dynamic, 16)
    for (i64 t = 0; t < T; ++t) {
        const uint8_t* a = targets + t * D;
        i64 best = -1, best_m = -1;
        for (i64 m = 0; m < M; ++m) {
            const uint8_t* b = neighbors + m * D;
            i64 s = 0;
            for (i64 d = 0; d < D; ++d) {
                const i64 e = (i64)a[d] - (i64)b[d];
                s += e * e;
            }
            if (best_m < 0 || s < best) {   /* strictly smaller: the lowest index wins ties */
                best = s;
                best_m = m;
            }
        }
        idx[t] = best_m;
        dist[t] = best;
    }
}
