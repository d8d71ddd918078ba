/*
 * rr_oracle.c -- plain CPU reference for the data-rearrangement operations of
 * "Fast GPGPU Data Rearrangement Kernels using CUDA" (Bader, Bungartz, Mudigere,
 * Narasimhan, Narayanan; arXiv:1011.3583).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle.  It shares no
 * code, header, table or helper with the GPU library; only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It is written
 * for obviousness, not speed: one loop over output elements, one odometer, one
 * memcpy per element.  No blocking, no fusion, no reordering.
 *
 * Semantics (what the paper computes, restated):
 *   Sec. III.B ("Data Re-ordering kernels"): an N-dimensional array stored
 *   linearly in row-major order is rewritten in another storage order given by
 *   a permutation of its axes.  Elements are opaque bytes; no arithmetic is done
 *   on values, so the result is unique and must match bit for bit.
 *   The paper writes orders fastest-dimension-first; this oracle offers both
 *   that notation (oracle_reorder_paper) and the row-major / NumPy notation
 *   (oracle_permute), so that the mapping between the two is itself checked.
 *
 *   The same section's N-to-M reorder (oracle_reorder_slice) reads a box of
 *   the input given by a base index and a range per dimension, keeps only the
 *   dimensions the order lists and fixes the others at their base.
 *
 *   Sec. III.A's read/write kernels move data by an access pattern: over a
 *   given set of indices (oracle_gather) or a given range (oracle_copy_range).
 *
 *   Sec. III.D's generic 2-D stencil (oracle_stencil2d) is the one operation
 *   that computes: a weighted sum of each point's neighbours, in double.
 *
 *   Sec. III.C ("Interlace, De-Interlace Kernels"): n equally long data sets are
 *   joined so that the set index varies fastest (interlace), or one such set is
 *   split back into n (de-interlace), e.g. complex numbers into real and
 *   imaginary planes.
 *
 * Build: gcc -O2 -shared -fPIC -o liboracle.so rr_oracle.c
 * A mutant build (-DRR_ORACLE_MUTANT=k, k>0) plants one deliberate mistake so
 * the tests can show that the pins catch it; it is never used for parity.
 */
#include <stdint.h>
#include <string.h>

#ifndef RR_ORACLE_MUTANT
#define RR_ORACLE_MUTANT 0
#endif

#define ORACLE_MAX_DIMS 16

/* Row-major strides (in elements): the last axis varies fastest. */
static void row_major_strides(int ndim, const int64_t* dims, int64_t* strides)
{
    int64_t s = 1;
    for (int k = ndim - 1; k >= 0; --k) {
        strides[k] = s;
#if RR_ORACLE_MUTANT == 3
        /* planted mistake: stride skips the fastest axis's extent */
        if (k != ndim - 1) s *= dims[k];
#else
        s *= dims[k];
#endif
    }
}

/*
 * Output element with output coordinates J (row-major over out_dims, where
 * out_dims[j] = dims[perm[j]]) is input element I with I[perm[j]] = J[j].
 * Return the input's linear element index.
 */
static int64_t source_index(int ndim, const int* perm, const int64_t* in_strides,
                            const int64_t* J)
{
    int64_t src = 0;
    for (int j = 0; j < ndim; ++j) {
#if RR_ORACLE_MUTANT == 1
        /* planted mistake: scatter instead of gather (uses the inverse perm) */
        int inv = 0;
        for (int k = 0; k < ndim; ++k) if (perm[k] == j) inv = k;
        src += J[j] * in_strides[inv];
#elif RR_ORACLE_MUTANT == 2
        /* planted mistake: drops the contribution of the slowest output axis */
        if (j == 0) continue;
        src += J[j] * in_strides[perm[j]];
#else
        src += J[j] * in_strides[perm[j]];
#endif
    }
    return src;
}

static int is_permutation(int ndim, const int* perm)
{
    int seen[ORACLE_MAX_DIMS] = {0};
    for (int j = 0; j < ndim; ++j) {
        if (perm[j] < 0 || perm[j] >= ndim || seen[perm[j]]) return 0;
        seen[perm[j]] = 1;
    }
    return 1;
}

/*
 * Permute (row-major / NumPy convention).
 *   dst has shape (dims[perm[0]], ..., dims[perm[ndim-1]]), row-major.
 *   dst[J] = src[I] with I[perm[j]] = J[j].
 * Returns 0 on success, -1 on bad arguments.
 */
int oracle_permute(void* dst, const void* src, int ndim, const int64_t* dims,
                   const int* perm, int esize)
{
    if (ndim < 1 || ndim > ORACLE_MAX_DIMS || esize < 1 || !is_permutation(ndim, perm))
        return -1;
    int64_t in_strides[ORACLE_MAX_DIMS];
    int64_t out_dims[ORACLE_MAX_DIMS];
    int64_t J[ORACLE_MAX_DIMS];
    int64_t total = 1;
    for (int k = 0; k < ndim; ++k) {
        if (dims[k] < 0) return -1;
        total *= dims[k];
    }
    if (total == 0) return 0;
    row_major_strides(ndim, dims, in_strides);
    for (int j = 0; j < ndim; ++j) { out_dims[j] = dims[perm[j]]; J[j] = 0; }

    unsigned char* d = (unsigned char*)dst;
    const unsigned char* s = (const unsigned char*)src;
    for (int64_t o = 0; o < total; ++o) {
        int64_t i = source_index(ndim, perm, in_strides, J);
        memcpy(d + o * esize, s + i * esize, (size_t)esize);
        /* odometer over output coordinates, last axis fastest */
        for (int j = ndim - 1; j >= 0; --j) {
            if (++J[j] < out_dims[j]) break;
            J[j] = 0;
        }
    }
    return 0;
}

/*
 * Permute, restricted to the output elements o_begin .. o_begin + o_count - 1
 * (the same definition as oracle_permute: dst[J] = src[I] with I[perm[j]] =
 * J[j]).  The odometer starts at the decoded coordinates of o_begin; dst holds
 * just those o_count elements.  Lets a test compute a huge output piece by
 * piece (and several pieces at once) without holding all of it.
 * Returns 0 on success, -1 on bad arguments or a range outside the output.
 */
int oracle_permute_range(void* dst, const void* src, int ndim, const int64_t* dims,
                         const int* perm, int esize, int64_t o_begin, int64_t o_count)
{
    if (ndim < 1 || ndim > ORACLE_MAX_DIMS || esize < 1 || !is_permutation(ndim, perm))
        return -1;
    int64_t in_strides[ORACLE_MAX_DIMS];
    int64_t out_dims[ORACLE_MAX_DIMS];
    int64_t J[ORACLE_MAX_DIMS];
    int64_t total = 1;
    for (int k = 0; k < ndim; ++k) {
        if (dims[k] < 0) return -1;
        total *= dims[k];
    }
    if (o_count < 0 || o_begin < 0 || o_begin > total || o_count > total - o_begin) return -1;
    if (o_count == 0) return 0;
    row_major_strides(ndim, dims, in_strides);
    for (int j = 0; j < ndim; ++j) out_dims[j] = dims[perm[j]];
    int64_t o = o_begin;
    for (int j = ndim - 1; j >= 0; --j) {   /* mixed-radix decode of the first index */
        J[j] = o % out_dims[j];
        o /= out_dims[j];
    }
    unsigned char* d = (unsigned char*)dst;
    const unsigned char* s = (const unsigned char*)src;
    for (int64_t t = 0; t < o_count; ++t) {
        int64_t i = source_index(ndim, perm, in_strides, J);
        memcpy(d + t * esize, s + i * esize, (size_t)esize);
        for (int j = ndim - 1; j >= 0; --j) {   /* odometer, last axis fastest */
            if (++J[j] < out_dims[j]) break;
            J[j] = 0;
        }
    }
    return 0;
}

/*
 * Same definition evaluated only at chosen output linear indices, for checking
 * huge outputs element by element.  out_index[t] is a linear index into dst;
 * the element's bytes go to samples + t*esize.
 */
int oracle_permute_at(void* samples, const void* src, int ndim, const int64_t* dims,
                      const int* perm, int esize, const int64_t* out_index, int64_t count)
{
    if (ndim < 1 || ndim > ORACLE_MAX_DIMS || esize < 1 || !is_permutation(ndim, perm))
        return -1;
    int64_t in_strides[ORACLE_MAX_DIMS];
    int64_t out_dims[ORACLE_MAX_DIMS];
    int64_t J[ORACLE_MAX_DIMS];
    int64_t total = 1;
    for (int k = 0; k < ndim; ++k) total *= dims[k];
    row_major_strides(ndim, dims, in_strides);
    for (int j = 0; j < ndim; ++j) out_dims[j] = dims[perm[j]];

    unsigned char* d = (unsigned char*)samples;
    const unsigned char* s = (const unsigned char*)src;
    for (int64_t t = 0; t < count; ++t) {
        int64_t o = out_index[t];
        if (o < 0 || o >= total) return -1;
        for (int j = ndim - 1; j >= 0; --j) {   /* mixed-radix decode */
            J[j] = o % out_dims[j];
            o /= out_dims[j];
        }
        int64_t i = source_index(ndim, perm, in_strides, J);
        memcpy(d + t * esize, s + i * esize, (size_t)esize);
    }
    return 0;
}

/*
 * Reorder in the paper's own notation (Sec. III.B): sizes[] and order[] are
 * listed fastest-changing dimension first.  Storage of the input: dimension 0
 * is fastest, so its linear index is sum_d x[d] * prod_{d'<d} sizes[d'].
 * The output's k-th fastest dimension is the input's dimension order[k]
 * (gather reading of "desired order").  The order [0 1 ... N-1] is a plain copy,
 * as the first row of the paper's Table 1 states.
 */
int oracle_reorder_paper(void* dst, const void* src, int ndim, const int64_t* sizes,
                         const int* order, int esize)
{
    if (ndim < 1 || ndim > ORACLE_MAX_DIMS || esize < 1 || !is_permutation(ndim, order))
        return -1;
    int64_t in_stride[ORACLE_MAX_DIMS];   /* fastest-first strides of the input */
    int64_t out_size[ORACLE_MAX_DIMS];    /* fastest-first extents of the output */
    int64_t K[ORACLE_MAX_DIMS];           /* output coordinates, fastest first  */
    int64_t total = 1;
    for (int d = 0; d < ndim; ++d) {
        if (sizes[d] < 0) return -1;
        in_stride[d] = total;
        total *= sizes[d];
    }
    if (total == 0) return 0;
    for (int k = 0; k < ndim; ++k) { out_size[k] = sizes[order[k]]; K[k] = 0; }

    unsigned char* dd = (unsigned char*)dst;
    const unsigned char* s = (const unsigned char*)src;
    for (int64_t o = 0; o < total; ++o) {
        int64_t i = 0;
        for (int k = 0; k < ndim; ++k) i += K[k] * in_stride[order[k]];
        memcpy(dd + o * esize, s + i * esize, (size_t)esize);
        for (int k = 0; k < ndim; ++k) {        /* odometer, dimension 0 fastest */
            if (++K[k] < out_size[k]) break;
            K[k] = 0;
        }
    }
    return 0;
}

/*
 * Interlace (Sec. III.C): n data sets of `count` elements each are joined into
 * one set in which the set index varies fastest:
 *   dst[i*n + c] = srcs[c][i],  0 <= i < count, 0 <= c < n.
 */
int oracle_interlace(void* dst, const void* const* srcs, int n, int64_t count, int esize)
{
    if (n < 1 || count < 0 || esize < 1) return -1;
    unsigned char* d = (unsigned char*)dst;
    for (int64_t i = 0; i < count; ++i) {
        for (int c = 0; c < n; ++c) {
            const unsigned char* s = (const unsigned char*)srcs[c];
#if RR_ORACLE_MUTANT == 4
            /* planted mistake: component-major instead of element-major */
            memcpy(d + (c * count + i) * esize, s + i * esize, (size_t)esize);
#else
            memcpy(d + (i * n + c) * esize, s + i * esize, (size_t)esize);
#endif
        }
    }
    return 0;
}

/*
 * De-interlace (Sec. III.C), the inverse split:
 *   dsts[c][i] = src[i*n + c].
 */
int oracle_deinterlace(void* const* dsts, const void* src, int n, int64_t count, int esize)
{
    if (n < 1 || count < 0 || esize < 1) return -1;
    const unsigned char* s = (const unsigned char*)src;
    for (int c = 0; c < n; ++c) {
        unsigned char* d = (unsigned char*)dsts[c];
        for (int64_t i = 0; i < count; ++i)
            memcpy(d + i * esize, s + (i * n + c) * esize, (size_t)esize);
    }
    return 0;
}

/*
 * N-to-M reorder with base and range (Sec. III.B: the reorder kernel's
 * N-to-M form keeps a base index and a range per dimension, and the output has
 * fewer dimensions than the input).  Row-major / NumPy convention:
 *   output axis j (0 <= j < out_ndim) runs over input axis order[j], from
 *   base[order[j]] for range[order[j]] steps; every input axis d that order
 *   does not list stays fixed at base[d].
 *   dst has shape (range[order[0]], ..., range[order[out_ndim-1]]), row-major;
 *   dst[J] = src[I] with I[order[j]] = base[order[j]] + J[j] and I[d] = base[d]
 *   for the other axes.
 * out_ndim = 0 copies the single element at base.  Returns 0 on success, -1 on
 * bad arguments (order not distinct, base or range outside dims).
 */
int oracle_reorder_slice(void* dst, const void* src, int ndim, const int64_t* dims,
                         const int64_t* base, const int64_t* range, int out_ndim,
                         const int* order, int esize)
{
    if (ndim < 1 || ndim > ORACLE_MAX_DIMS || out_ndim < 0 || out_ndim > ndim || esize < 1) return -1;
    int kept[ORACLE_MAX_DIMS] = {0};
    for (int j = 0; j < out_ndim; ++j) {
        if (order[j] < 0 || order[j] >= ndim || kept[order[j]]) return -1;
        kept[order[j]] = 1;
    }
    for (int d = 0; d < ndim; ++d) {
        if (dims[d] < 0 || base[d] < 0) return -1;
        if (kept[d]) {
            if (range[d] < 0 || base[d] + range[d] > dims[d]) return -1;
        } else if (base[d] >= dims[d]) {
            return -1;
        }
    }
    int64_t in_strides[ORACLE_MAX_DIMS];
    row_major_strides(ndim, dims, in_strides);
    /* offset of the element every output element starts from: the fixed axes
       at their base, the kept axes at the start of their range */
    int64_t start = 0;
    for (int d = 0; d < ndim; ++d) {
#if RR_ORACLE_MUTANT == 5
        /* planted mistake: fixed axes read at index 0 instead of their base */
        if (!kept[d]) continue;
#elif RR_ORACLE_MUTANT == 6
        /* planted mistake: kept axes start at 0 instead of their base */
        if (kept[d]) continue;
#endif
        start += base[d] * in_strides[d];
    }
    int64_t out_dims[ORACLE_MAX_DIMS];
    int64_t J[ORACLE_MAX_DIMS];
    int64_t total = 1;
    for (int j = 0; j < out_ndim; ++j) { out_dims[j] = range[order[j]]; J[j] = 0; total *= out_dims[j]; }
    if (total == 0) return 0;

    unsigned char* o = (unsigned char*)dst;
    const unsigned char* s = (const unsigned char*)src;
    for (int64_t t = 0; t < total; ++t) {
        int64_t i = start;
        for (int j = 0; j < out_ndim; ++j) i += J[j] * in_strides[order[j]];
        memcpy(o + t * esize, s + i * esize, (size_t)esize);
        for (int j = out_ndim - 1; j >= 0; --j) {
            if (++J[j] < out_dims[j]) break;
            J[j] = 0;
        }
    }
    return 0;
}

/*
 * Read kernel over an index set (Sec. III.A: the read/write kernels take access
 * patterns such as a given set of indices): dst[i] = src[idx[i]] for
 * 0 <= i < count.  Indices outside [0, src_count) are rejected (-1).
 */
int oracle_gather(void* dst, const void* src, int64_t src_count, const int64_t* idx, int64_t count,
                  int esize)
{
    if (count < 0 || src_count < 0 || esize < 1) return -1;
    for (int64_t i = 0; i < count; ++i)
        if (idx[i] < 0 || idx[i] >= src_count) return -1;
    unsigned char* d = (unsigned char*)dst;
    const unsigned char* s = (const unsigned char*)src;
    for (int64_t i = 0; i < count; ++i) {
#if RR_ORACLE_MUTANT == 7
        /* planted mistake: reads the index array one position late */
        int64_t k = (i + 1 < count) ? idx[i + 1] : idx[i];
        memcpy(d + i * esize, s + k * esize, (size_t)esize);
#else
        memcpy(d + i * esize, s + idx[i] * esize, (size_t)esize);
#endif
    }
    return 0;
}

/*
 * Read kernel over a range (Sec. III.A: access based on a specified range):
 * dst[i] = src[start + i*stride] for 0 <= i < count (stride may be negative or
 * zero).  Every read index must lie in [0, src_count), else -1.
 */
int oracle_copy_range(void* dst, const void* src, int64_t src_count, int64_t start, int64_t stride,
                      int64_t count, int esize)
{
    if (count < 0 || src_count < 0 || esize < 1) return -1;
    if (count == 0) return 0;
    int64_t last = start + (count - 1) * stride;
    if (start < 0 || start >= src_count || last < 0 || last >= src_count) return -1;
    unsigned char* d = (unsigned char*)dst;
    const unsigned char* s = (const unsigned char*)src;
    for (int64_t i = 0; i < count; ++i) {
#if RR_ORACLE_MUTANT == 8
        /* planted mistake: ignores the start of the range */
        int64_t k = i * stride + (stride < 0 ? start : 0);
#else
        int64_t k = start + i * stride;
#endif
        memcpy(d + i * esize, s + k * esize, (size_t)esize);
    }
    return 0;
}

/*
 * 2-D stencil (Sec. III.D: each grid point is updated with weighted
 * contributions of its neighbours; the measured case is a finite-difference
 * stencil of orders I-IV on single-precision data).  Evaluated in double from
 * float inputs and float weights, in the order written here.
 *   src, dst: rows x cols floats, row-major.  radius r in 1..4.
 *   shape 0 (star): weights[0..r]; out = w0*x[i][j] + sum_{k=1..r} wk *
 *     (x[i-k][j] + x[i+k][j] + x[i][j-k] + x[i][j+k]).
 *   shape 1 (box): weights[(2r+1)^2], row-major over dy = -r..r, dx = -r..r;
 *     out = sum w[dy][dx] * x[i+dy][j+dx].
 *   Points closer than r to an edge keep their input value.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_stencil2d(double* dst, const float* src, int64_t rows, int64_t cols, int radius, int shape,
                     const float* weights)
{
    if (rows < 0 || cols < 0 || radius < 1 || radius > 4 || (shape != 0 && shape != 1)) return -1;
    const int r = radius;
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            const float* x = src + i * cols + j;
            if (i < r || i >= rows - r || j < r || j >= cols - r) {
                dst[i * cols + j] = (double)*x;
                continue;
            }
            double acc = 0.0;
            if (shape == 0) {
                acc = (double)weights[0] * (double)x[0];
                for (int k = 1; k <= r; ++k) {
#if RR_ORACLE_MUTANT == 9
                    /* planted mistake: the vertical neighbours use the horizontal offset */
                    double ring = (double)x[-k] + (double)x[k] + (double)x[-k] + (double)x[k];
#else
                    double ring = (double)x[-k * cols] + (double)x[k * cols] + (double)x[-k] + (double)x[k];
#endif
                    acc += (double)weights[k] * ring;
                }
            } else {
                const int n = 2 * r + 1;
                for (int dy = -r; dy <= r; ++dy)
                    for (int dx = -r; dx <= r; ++dx)
                        acc += (double)weights[(dy + r) * n + (dx + r)] * (double)x[dy * cols + dx];
            }
            dst[i * cols + j] = acc;
        }
    }
    return 0;
}

/* Identity of the build, so a test can tell a mutant from the real oracle. */
int oracle_mutant_id(void) { return RR_ORACLE_MUTANT; }
