/*
 * Oracle for hashless content-defined chunking (RAM, AE-Max, AE-Min, MAXP).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition that the GPU path is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links or calls it, and it shares no code, header or
 * constant with the HIP sources.
 *
 * Every chunker is written as the native, byte-at-a-time loop the paper
 * describes (the accelerated versions must reproduce these cuts exactly,
 * Section 6.1, "Vector-acceleration Impact").  Conventions shared by all:
 *
 *   x[0..n)   bytes, compared as UNSIGNED values (Section 4.1: 0xE1 is the
 *             maximum of 0xE1 and 0x21).
 *   w >= 1    window size; M >= w+1 maximum chunk size.
 *   driver    s = 0; while s < n: c = next(s); emit c; s = c.
 *             Emitted values are exclusive chunk ends; the last one is n.
 *   L(s)      min(n, s+M): the hard limit of the chunk that starts at s
 *             (a forced cut at the maximum chunk size).
 *
 * Readings of the prose (where it is silent or ambiguous) are listed with
 * each next() function.
 */
#include <stdint.h>
#include <stddef.h>

#define ORACLE_ALGO_RAM 0
#define ORACLE_ALGO_AE_MAX 1
#define ORACLE_ALGO_MAXP 2
#define ORACLE_ALGO_AE_MIN 3

static uint64_t lim(uint64_t s, uint64_t n, uint64_t M) {
    return (n - s > M) ? s + M : n;
}

/*
 * RAM (Section 2.1 "RAM", Fig. 2c; Section 4.3).
 * The maximum T of the fixed window at the start of the chunk, x[s..s+w),
 * is found first (an extreme byte search); scanning then starts at the first
 * byte outside the window, and the chunk ends at the first byte that is
 * greater than or equal to T (a range scan with GEQ).  Reading: the chunk
 * includes that byte, so the cut is j+1.  If the window does not fit before
 * the limit, or no such byte exists before the limit, the cut is the limit.
 */
static uint64_t next_ram(const uint8_t* x, uint64_t n, uint64_t w, uint64_t M,
                         uint64_t s) {
    uint64_t L = lim(s, n, M);
    if (s + w >= L) return L;
    uint8_t T = 0;
    for (uint64_t i = s; i < s + w; i++)
        if (x[i] > T) T = x[i];
    for (uint64_t j = s + w; j < L; j++)
        if (x[j] >= T) return j + 1;
    return L;
}

/*
 * AE-Max (Section 2.1 "AE", Fig. 2a; Section 4.3).
 * A target is a byte greater than every byte before it in the chunk; the
 * chunk's first byte trivially is one.  If no byte in the w bytes after the
 * target is greater than the target, the cut goes right after that window
 * (at p+w+1); otherwise the first greater byte becomes the new target.
 * Reading of ties: new targets are found with the GT comparator, so a window
 * byte equal to the target neither becomes a target nor blocks the cut.
 */
static uint64_t next_ae_max(const uint8_t* x, uint64_t n, uint64_t w,
                            uint64_t M, uint64_t s) {
    uint64_t L = lim(s, n, M);
    uint64_t p = s;
    for (uint64_t i = s + 1; i < L; i++) {
        if (x[i] > x[p])
            p = i;
        else if (i == p + w)
            return i + 1;
    }
    return L;
}

/* AE-Min (Section 2.1 "AE"; Section 4.3): AE-Max with minima (LT). */
static uint64_t next_ae_min(const uint8_t* x, uint64_t n, uint64_t w,
                            uint64_t M, uint64_t s) {
    uint64_t L = lim(s, n, M);
    uint64_t p = s;
    for (uint64_t i = s + 1; i < L; i++) {
        if (x[i] < x[p])
            p = i;
        else if (i == p + w)
            return i + 1;
    }
    return L;
}

/* Strict local maximum: x[i] is greater than each of the w bytes before it
 * and each of the w bytes after it (Section 2.1 "MAXP", Fig. 2b). */
static int strict_local_max(const uint8_t* x, uint64_t i, uint64_t w) {
    for (uint64_t j = i - w; j < i; j++)
        if (x[j] >= x[i]) return 0;
    for (uint64_t j = i + 1; j <= i + w; j++)
        if (x[j] >= x[i]) return 0;
    return 1;
}

/*
 * MAXP (Section 2.1 "MAXP", Fig. 2b; Section 4.3).
 * Two windows of w bytes slide over the data one byte apart; the byte
 * between them is the target.  When the target is greater than the maximum
 * of both windows, the chunk ends right after it (cut i+1).  Readings: the
 * left window lies inside the chunk (targets start at s+w); the right window
 * must be complete (i+w <= n-1); only the target, not its right window, is
 * bounded by the chunk limit.
 */
static uint64_t next_maxp(const uint8_t* x, uint64_t n, uint64_t w, uint64_t M,
                          uint64_t s) {
    uint64_t L = lim(s, n, M);
    for (uint64_t i = s + w; i < L; i++) {
        if (i + w >= n) break;
        if (strict_local_max(x, i, w)) return i + 1;
    }
    return L;
}

static int params_ok(uint64_t w, uint64_t M) { return w >= 1 && M >= w + 1; }

/* One step of the chain: the exclusive end of the chunk starting at s. */
uint64_t oracle_next(int algo, const uint8_t* x, uint64_t n, uint64_t w,
                     uint64_t M, uint64_t s) {
    switch (algo) {
        case ORACLE_ALGO_RAM: return next_ram(x, n, w, M, s);
        case ORACLE_ALGO_AE_MAX: return next_ae_max(x, n, w, M, s);
        case ORACLE_ALGO_MAXP: return next_maxp(x, n, w, M, s);
        case ORACLE_ALGO_AE_MIN: return next_ae_min(x, n, w, M, s);
    }
    return 0;
}

/*
 * Chunk x[0..n) and write the exclusive chunk ends to cuts[0..cap).
 * Returns the number of cuts, -1 for invalid parameters, -2 if cap is too
 * small (the cuts written so far are valid).
 */
int64_t oracle_chunk(int algo, const uint8_t* x, uint64_t n, uint64_t w,
                     uint64_t M, uint64_t* cuts, uint64_t cap) {
    if (!params_ok(w, M) || algo < 0 || algo > 3) return -1;
    uint64_t k = 0, s = 0;
    while (s < n) {
        uint64_t c = oracle_next(algo, x, n, w, M, s);
        if (k == cap) return -2;
        cuts[k++] = c;
        s = c;
    }
    return (int64_t)k;
}

/*
 * Many buffers of one byte array, each chunked on its own by the driver of
 * oracle_chunk: buffer j is x[off[j] .. off[j] + len[j]); its cuts go to
 * cuts[base[j] ..) (room for (len-1)/(w+1)+1 values) and their number to
 * counts[j].  Returns 0, or the first negative status of oracle_chunk.
 */
int64_t oracle_chunk_many(int algo, const uint8_t* x, const uint64_t* off,
                          const uint64_t* len, uint64_t njobs, uint64_t w,
                          uint64_t M, uint64_t* cuts, const uint64_t* base,
                          int64_t* counts) {
    for (uint64_t j = 0; j < njobs; j++) {
        uint64_t room = len[j] == 0 ? 0 : (len[j] - 1) / (w + 1) + 1;
        int64_t k = oracle_chunk(algo, x + off[j], len[j], w, M,
                                 cuts + base[j], room);
        if (k < 0) return k;
        counts[j] = k;
    }
    return 0;
}

/*
 * Bytes per pattern (Section 6.3 measures the share of bytes each pattern
 * handles: RAM spends nearly all of them in the extreme byte search, MAXP in
 * the range scan).  The chain is the one oracle_chunk computes; each chunk
 * [s, c) is split by the way Section 4.3 builds the chunker from the two
 * patterns:
 *   RAM     the window [s, min(s+w, c)) is searched for its maximum (EBS);
 *           the bytes after it up to the cut are range-scanned (RS).
 *   AE      bytes up to and including the final target p (the targets are
 *           found by range scans) are RS; the bytes after p up to the cut
 *           are the window whose maximum is compared with p (EBS).
 *   MAXP    a content cut after the target i = c-1 searches both windows of
 *           i, 2w bytes (EBS; the right one lies past the cut); the other
 *           bytes of the chunk, those before the left window and the target
 *           itself, are range-scanned (RS).  A forced or final chunk is all
 *           RS.
 * out[0] += EBS bytes, out[1] += RS bytes.  Returns the number of chunks, or
 * -1 for invalid parameters.
 */
int64_t oracle_pattern_bytes(int algo, const uint8_t* x, uint64_t n, uint64_t w,
                             uint64_t M, uint64_t* out) {
    if (!params_ok(w, M) || algo < 0 || algo > 3) return -1;
    int64_t k = 0;
    uint64_t s = 0;
    while (s < n) {
        uint64_t c = oracle_next(algo, x, n, w, M, s);
        uint64_t len = c - s;
        if (algo == ORACLE_ALGO_RAM) {
            uint64_t win = len < w ? len : w;
            out[0] += win;
            out[1] += len - win;
        } else if (algo == ORACLE_ALGO_AE_MAX || algo == ORACLE_ALGO_AE_MIN) {
            /* the final target: the last record before the cut */
            uint64_t p = s;
            for (uint64_t i = s + 1; i < c; i++) {
                int better = algo == ORACLE_ALGO_AE_MAX ? x[i] > x[p] : x[i] < x[p];
                if (better) p = i;
            }
            out[1] += p - s + 1;
            out[0] += c - p - 1;
        } else {
            /* a content cut: c-1 is a strict local maximum with full windows
               and at least w bytes into its chunk */
            uint64_t i = c - 1;
            if (i >= s + w && i + w < n && strict_local_max(x, i, w)) {
                out[0] += 2 * w;
                out[1] += len - w;
            } else {
                out[1] += len;
            }
        }
        k++;
        s = c;
    }
    return k;
}
