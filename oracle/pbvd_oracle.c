/*
 * pbvd_oracle.c -- plain CPU oracle for the parallel block-based Viterbi
 * decoder (PBVD) of Peng, Liu, Hou and Zhao, "A Gb/s Parallel Block-based
 * Viterbi Decoder for Convolutional Codes on GPU" (arXiv 1608.00066).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it, as the reference the GPU decoder is compared
 * against bit for bit.
 *
 * It is deliberately slow and literal: int64 path metrics, one byte per
 * survivor decision, no SIMD, no blocking beyond the one the method itself
 * defines.  It shares no code, header, table or constant with the GPU
 * library.
 *
 * Readings of points the paper leaves open are listed next to the code they
 * affect and are the same ones the design document lists:
 *   - generator bit k of gen[r] is g_k^(r) of Eq. 2; bit K-1 taps the input x;
 *   - state d = (D_{K-2} ... D_0)_2, D_{K-2} holds the newest input bit
 *     (the butterfly of Sec. III-B: S_2j, S_2j+1 -> S_j for x=0 and
 *     S_{j+2^{K-2}} for x=1);
 *   - an encoder output c = [c^(1) ... c^(R)] is packed as an integer with
 *     c^(1) as its most significant bit;
 *   - branch metric = sum over the R symbols of |q| where the hard sign of q
 *     disagrees with the code bit (q >= 0 reads as bit 0);
 *   - ties in add-compare-select keep the upper branch (from S_2j);
 *   - a block whose forward range starts at stage 0 starts from the known
 *     encoder state 0 (other states get ORACLE_BIG); every other block starts
 *     from all-zero metrics, as Sec. III-A prescribes;
 *   - traceback starts from state 0 (Sec. III-A, Alg. 1), except at the end
 *     of an unterminated stream, where it starts from the state of minimum
 *     path metric (lowest index on ties), as in full-frame Viterbi (Sec. II);
 *   - the block geometry at the two stream ends is clipped to [0, T).
 *
 * Parity status: every function below is pinned by tests that do not reuse
 * its arithmetic (Table II, Eq. 3-6 identities, impulse responses, free
 * distances, brute-force maximum likelihood, noiseless decoding, block versus
 * full-frame equivalence, split invariance).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_BIG 8192
#define ORACLE_MAX_K 12
#define ORACLE_MAX_R 8

enum { ORACLE_SOFT_I8 = 0, ORACLE_HARD_U8 = 1 };

static int parity_u32(uint32_t x)
{
    int p = 0;
    while (x) {
        p ^= 1;
        x &= x - 1;
    }
    return p;
}

/* Eq. 2: c^(r) = x*g_{K-1} xor D_{K-2}*g_{K-2} xor ... xor D_0*g_0.
 * The shift register holds x in bit K-1 and D_k in bit k, so every code bit
 * is the parity of (register AND generator). */
static int encoder_output(int K, int R, const uint32_t *gen, int d, int x)
{
    uint32_t reg = ((uint32_t)x << (K - 1)) | (uint32_t)d;
    int c = 0;
    for (int r = 0; r < R; r++)
        c = (c << 1) | parity_u32(reg & gen[r]);
    return c;
}

/* Butterfly of Sec. III-B: input x moves S_d to S_{(x << (K-2)) | (d >> 1)}. */
static int next_state(int K, int d, int x)
{
    return (x << (K - 2)) | (d >> 1);
}

static int check_code(int K, int R, const uint32_t *gen)
{
    if (K < 2 || K > ORACLE_MAX_K || R < 1 || R > ORACLE_MAX_R || !gen)
        return -1;
    for (int r = 0; r < R; r++)
        if (gen[r] >> K)
            return -1;
    return 0;
}

/* Trellis tables: next[d][x] and the packed encoder output label[d][x]
 * for every state d and input x (Eq. 2 and the butterfly of Sec. III-B). */
int oracle_trellis(int K, int R, const uint32_t *gen, int32_t *next, int32_t *label)
{
    if (check_code(K, R, gen))
        return -1;
    int N = 1 << (K - 1);
    for (int d = 0; d < N; d++)
        for (int x = 0; x < 2; x++) {
            if (next)
                next[2 * d + x] = next_state(K, d, x);
            if (label)
                label[2 * d + x] = encoder_output(K, R, gen, d, x);
        }
    return 0;
}

/* Received value of one code symbol: a signed int8 soft value, or a hard
 * bit mapped to +1 (bit 0) / -1 (bit 1) so that the metric below becomes the
 * Hamming distance (Sec. II names Hamming and Euclidean distance). */
static int64_t received_value(int input_kind, uint8_t byte)
{
    if (input_kind == ORACLE_HARD_U8)
        return 1 - 2 * (int64_t)(byte & 1);
    return (int64_t)(int8_t)byte;
}

/* Branch metric of Sec. II: the distance between the received symbols of
 * one stage and code word c.  A code bit costs |q| when it disagrees with
 * the sign of q (q >= 0 means bit 0), and nothing otherwise. */
static int64_t branch_metric(int R, int input_kind, const uint8_t *stage_syms, int c)
{
    int64_t bm = 0;
    for (int r = 0; r < R; r++) {
        int code_bit = (c >> (R - 1 - r)) & 1;
        int64_t q = received_value(input_kind, stage_syms[r]);
        int hard = q < 0;
        if (code_bit != hard)
            bm += q < 0 ? -q : q;
    }
    return bm;
}

/* All 2^R branch metrics of stages [0, n_stages): bm[s][c]. */
int oracle_branch_metrics(int R, int input_kind, const uint8_t *syms, int64_t n_stages, int64_t *bm)
{
    if (R < 1 || R > ORACLE_MAX_R || n_stages < 0 || (n_stages && (!syms || !bm)))
        return -1;
    if (input_kind != ORACLE_SOFT_I8 && input_kind != ORACLE_HARD_U8)
        return -1;
    int C = 1 << R;
    for (int64_t s = 0; s < n_stages; s++)
        for (int c = 0; c < C; c++)
            bm[s * C + c] = branch_metric(R, input_kind, syms + s * R, c);
    return 0;
}

/* Number of parallel blocks of Sec. III-A for n decoded bits: ceil(n / D). */
int64_t oracle_num_blocks(int64_t n, int64_t D)
{
    if (n < 1 || D < 1)
        return 0;
    return (n + D - 1) / D;
}

/* Geometry of parallel block b (Sec. III-A, Fig. 1 and 2, M = L): the
 * forward range [t - L, t + D + L) with t = b*D, clipped to the T trellis
 * stages, and the decoded range [t, t + D) clipped to the n information bits.
 * out = {f0, f1, d0, d1}. */
void oracle_pb_geometry(int64_t n, int64_t T, int64_t D, int64_t L, int64_t b, int64_t *out)
{
    int64_t t = b * D;
    int64_t f0 = t - L;
    int64_t f1 = t + D + L;
    int64_t d1 = t + D;
    out[0] = f0 < 0 ? 0 : f0;
    out[1] = f1 > T ? T : f1;
    out[2] = t;
    out[3] = d1 > n ? n : d1;
}

struct oracle_job {
    int K, R, D, L, terminated, input_kind;
    const uint32_t *gen;
    const uint8_t *syms;
    int64_t n, T, pb_first, pb_count;
    uint8_t *bits;
    int64_t *final_pm;
    uint8_t *dec_out;
    int64_t next_pb;
    pthread_mutex_t lock;
    int failed;
};

/* Decode one parallel block: forward add-compare-select over its whole
 * forward range (Eq. 1, Sec. III-A), then traceback from the start state
 * along the stored survivors, emitting the bits of its decoded range. */
static int decode_block(struct oracle_job *job, int64_t b, int64_t *pm, int64_t *pm_next, uint8_t *dec)
{
    const int K = job->K, R = job->R;
    const int N = 1 << (K - 1);
    int32_t next[2 << ORACLE_MAX_K], label[2 << ORACLE_MAX_K];
    oracle_trellis(K, R, job->gen, next, label);

    int64_t g[4];
    oracle_pb_geometry(job->n, job->T, job->D, job->L, b, g);
    const int64_t f0 = g[0], f1 = g[1], d0 = g[2], d1 = g[3];

    /* Initial metrics: the encoder starts in state 0, so a block that
     * starts at stage 0 knows its state; any other block starts from the
     * unknown state with all metrics zero (Sec. III-A). */
    for (int d = 0; d < N; d++)
        pm[d] = (f0 == 0 && d != 0) ? ORACLE_BIG : 0;

    /* Forward procedure: Eq. 1, PM_n^j = min_i (PM_{n-1}^i + BM_n^{i,j}).
     * State j has the two predecessors i = 2*(j mod 2^{K-2}) (upper branch)
     * and i + 1 (lower branch); the decision bit is 1 for the lower one. */
    for (int64_t s = f0; s < f1; s++) {
        const uint8_t *q = job->syms + s * R;
        for (int j = 0; j < N; j++) {
            int x = j >> (K - 2);
            int i_up = 2 * (j & ((N >> 1) - 1));
            int i_lo = i_up + 1;
            int64_t a = pm[i_up] + branch_metric(R, job->input_kind, q, label[2 * i_up + x]);
            int64_t c = pm[i_lo] + branch_metric(R, job->input_kind, q, label[2 * i_lo + x]);
            if (next[2 * i_up + x] != j || next[2 * i_lo + x] != j)
                return -1; /* the butterfly and the transition table disagree */
            int lower = c < a; /* ties keep the upper branch */
            dec[(s - f0) * N + j] = (uint8_t)lower;
            pm_next[j] = lower ? c : a;
        }
        memcpy(pm, pm_next, sizeof(int64_t) * N);
    }

    int64_t pm_min = pm[0];
    int argmin = 0;
    for (int d = 1; d < N; d++)
        if (pm[d] < pm_min) {
            pm_min = pm[d];
            argmin = d;
        }

    int64_t local = b - job->pb_first;
    if (job->final_pm)
        for (int d = 0; d < N; d++)
            job->final_pm[local * N + d] = pm[d] - pm_min;

    if (job->dec_out) {
        /* decisions of stages [d0, f1), row s - d0, state-indexed */
        uint8_t *dst = job->dec_out + local * (int64_t)(job->D + job->L) * N;
        memset(dst, 0, (size_t)(job->D + job->L) * N);
        for (int64_t s = d0; s < f1; s++)
            memcpy(dst + (s - d0) * N, dec + (s - f0) * N, N);
    }

    /* Traceback (Sec. III-A, Alg. 1): start from state 0, or, at the end of
     * an unterminated stream, from the best state as in full-frame Viterbi;
     * walk back to the start of the decoded range; the input bit that led
     * into a state is its top bit. */
    int state = (f1 == job->T && !job->terminated) ? argmin : 0;
    for (int64_t s = f1 - 1; s >= d0; s--) {
        if (s < d1)
            job->bits[s - job->pb_first * job->D] = (uint8_t)((state >> (K - 2)) & 1);
        int lower = dec[(s - f0) * N + state];
        state = 2 * (state & ((N >> 1) - 1)) + lower;
    }
    return 0;
}

static void *worker(void *arg)
{
    struct oracle_job *job = (struct oracle_job *)arg;
    const int N = 1 << (job->K - 1);
    int64_t span = (int64_t)job->D + 2 * (int64_t)job->L;
    if (span > job->T)
        span = job->T;
    int64_t *pm = malloc(sizeof(int64_t) * N);
    int64_t *pm_next = malloc(sizeof(int64_t) * N);
    uint8_t *dec = malloc((size_t)span * N + 1);
    if (!pm || !pm_next || !dec) {
        pthread_mutex_lock(&job->lock);
        job->failed = 1;
        pthread_mutex_unlock(&job->lock);
    } else {
        for (;;) {
            pthread_mutex_lock(&job->lock);
            int64_t b = job->next_pb++;
            int stop = job->failed;
            pthread_mutex_unlock(&job->lock);
            if (stop || b >= job->pb_first + job->pb_count)
                break;
            if (decode_block(job, b, pm, pm_next, dec)) {
                pthread_mutex_lock(&job->lock);
                job->failed = 1;
                pthread_mutex_unlock(&job->lock);
                break;
            }
        }
    }
    free(pm);
    free(pm_next);
    free(dec);
    return NULL;
}

/*
 * Block-based decode of parallel blocks [pb_first, pb_first + pb_count) of a
 * stream of n information bits (Sec. III-A).
 *   syms      : T*R received symbols, stage-major (T = n + (K-1)*terminated)
 *   bits      : one byte (0/1) per decoded bit, indexed from bit pb_first*D
 *   final_pm  : [pb_count][N] metrics at the end of each block minus their
 *               minimum, or NULL
 *   dec_out   : [pb_count][D+L][N] decisions of stages [b*D, f1), or NULL
 *   nthreads  : worker threads over blocks (1 = single-threaded)
 * Full-frame Viterbi (Sec. II) is the case D >= n.
 * Returns 0, or -1 on invalid arguments or allocation failure.
 */
int oracle_decode(int K, int R, const uint32_t *gen, int D, int L, int terminated, int input_kind,
                  const uint8_t *syms, int64_t n, int64_t pb_first, int64_t pb_count, uint8_t *bits,
                  int64_t *final_pm, uint8_t *dec_out, int nthreads)
{
    if (check_code(K, R, gen) || D < 1 || L < 0 || n < 1 || !syms || !bits)
        return -1;
    if (input_kind != ORACLE_SOFT_I8 && input_kind != ORACLE_HARD_U8)
        return -1;
    int64_t nb = oracle_num_blocks(n, D);
    if (pb_first < 0 || pb_count < 0 || pb_first + pb_count > nb)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;

    struct oracle_job job;
    memset(&job, 0, sizeof(job));
    job.K = K;
    job.R = R;
    job.D = D;
    job.L = L;
    job.terminated = terminated ? 1 : 0;
    job.input_kind = input_kind;
    job.gen = gen;
    job.syms = syms;
    job.n = n;
    job.T = n + (terminated ? K - 1 : 0);
    job.pb_first = pb_first;
    job.pb_count = pb_count;
    job.bits = bits;
    job.final_pm = final_pm;
    job.dec_out = dec_out;
    job.next_pb = pb_first;
    pthread_mutex_init(&job.lock, NULL);

    if (nthreads == 1) {
        worker(&job);
    } else {
        pthread_t tid[256];
        int started = 0;
        for (int t = 0; t < nthreads; t++) {
            if (pthread_create(&tid[t], NULL, worker, &job))
                break;
            started++;
        }
        if (!started)
            worker(&job);
        for (int t = 0; t < started; t++)
            pthread_join(tid[t], NULL);
    }
    pthread_mutex_destroy(&job.lock);
    return job.failed ? -1 : 0;
}
