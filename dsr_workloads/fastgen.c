/* Fast path of the input generator: splitmix64 draws mapped to fp32
 * uniform on [-1, 1), the same definition as gen.py (draw n of a stream is
 * the n-th output of splitmix64 started at the stream's base state; fp32 =
 * (u >> 40) * 2^-23 - 1).  Threads split the index range. */
#include <pthread.h>
#include <stdint.h>

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t dsrgen_stream_base(uint64_t seed, uint64_t stream)
{
    return mix64(seed ^ (stream * 0xD1B54A32D192ED03ull));
}

typedef struct { uint64_t base, start, count; float *out; } job_t;

static void *run(void *p)
{
    job_t *j = (job_t *)p;
    for (uint64_t k = 0; k < j->count; ++k) {
        uint64_t u = mix64(j->base + (j->start + k + 1) * 0x9E3779B97F4A7C15ull);
        j->out[k] = (float)((double)(u >> 40) * 0x1p-23 - 1.0);
    }
    return 0;
}

void dsrgen_f32(uint64_t seed, uint64_t stream, uint64_t start, uint64_t count, float *out,
                int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    if (count < (1u << 20)) threads = 1;
    pthread_t th[64];
    job_t jobs[64];
    const uint64_t base = dsrgen_stream_base(seed, stream);
    const uint64_t per = (count + threads - 1) / threads;
    for (int t = 0; t < threads; ++t) {
        uint64_t lo = per * t < count ? per * t : count;
        uint64_t hi = lo + per < count ? lo + per : count;
        jobs[t].base = base;
        jobs[t].start = start + lo;
        jobs[t].count = hi - lo;
        jobs[t].out = out + lo;
        if (t) pthread_create(&th[t], 0, run, &jobs[t]);
    }
    run(&jobs[0]);
    for (int t = 1; t < threads; ++t) pthread_join(th[t], 0);
}
