// lap_scalar.hpp -- the Hungarian LAP solver of lap_wave.hpp with its control
// held in scalar registers: a wavefront solves one LAP on 64 lanes (m <= 64,
// lap_solve_scalar1) or two on 32 lanes each (m <= 32, lap_solve_scalar2).
// Lane l of a part owns row l and column l of its LAP.
//
// Same algorithm, same arithmetic, same tie-break as lap_wave.hpp (column
// reduction start, then shortest augmenting paths, Section 2.3 "LAP
// Solution"; see there for the fixed choice of optimal duals), so results are
// bitwise identical.  What differs is the mapping: the current row, the
// chosen column, the matched row and the path are wave-uniform values in
// SGPRs, and the per-column flags (tree rows, tree columns, unmatched
// columns) are wave masks there too, so the scalar unit runs the control
// flow and a Dijkstra step costs about thirty-three vector instructions.
//
// Data: the block's LDS array `lds` holds a part's matrix (row stride m) at
// lds + tile offset and its scratch at lds + scratch offset (m doubles: row
// potentials, then m ints: matching, then m ints: proposals).  Offsets rather
// than pointers keep every access a known LDS access (a per-lane choice
// between generic pointers compiles to flat loads).  Outputs for lane l of a
// part: u (row l), v (column l), p (row matched to column l, -1 past m);
// theta and steps of the lane's part.  On return the scratch holds the
// part's row potentials.
#pragma once
#include <hip/hip_runtime.h>

#include "lap_wave.hpp"

namespace qap {

// Sixteen (eight) doubles per lane, indexed by a wave-uniform row in
// registers.
typedef double dreg16 __attribute__((ext_vector_type(16)));
typedef double dreg8 __attribute__((ext_vector_type(8)));


// A copy of x in its own register pair, made by one 64-bit move (the
// permlane swaps below overwrite both of their operands, and a copy of the
// two 32-bit halves takes two moves).
__device__ __forceinline__ double vcopy_d(double x)
{
    asm("" : "+v"(x));
    return x;
}

// min over each 16-lane row (RW = 16), each 32-lane half (RW = 32) or the
// whole wave (RW = 64); every lane receives the minimum of its row / half /
// wave.  The solvers call it with RW no smaller than the lanes their live
// columns span, so the lanes that matter get the part's minimum; the others
// hold +inf or NaN and are never chosen.
template <int RW>
__device__ __forceinline__ double part_min(double x)
{
    x = dmin(x, dpp_d<0x128>(x));  // row_ror:8
    x = dmin(x, dpp_d<0x124>(x));  // row_ror:4
    x = dmin(x, dpp_d<0x122>(x));  // row_ror:2
    x = dmin(x, dpp_d<0x121>(x));  // row_ror:1
    if constexpr (RW >= 32) {
        const double y = vcopy_d(x);
        const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
        x = dmin(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
    }
    if constexpr (RW == 64) {
        const double y = vcopy_d(x);
        const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
        x = dmin(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
    }
    return x;
}

// One LAP per wavefront with the per-column flags held as wave masks in
// SGPRs rather than per-lane booleans: the tree rows, the tree (used)
// columns and the unmatched columns.  A mask turns back into
// a lane predicate for free (inverse ballot: the SGPR pair is the lane mask
// of a v_cndmask or of exec), so the tie-break ballot is a single compare
// and the flag updates are scalar bit operations.  Non-tree valid columns
// keep minv, every other lane holds +inf, so the step's minimum reads minv
// directly.
// Tile at lds + toff, scratch at lds + soff; m <= RW (RW = 32 or 16: every
// live column sits in the lowest 32 or 16 lanes and the minimum stops
// there).
//
// KR > 0 (KR <= m, KR <= 24): rows 0..KR-1 of the tile are held in
// registers instead, lane l holding entry (r, l) of row r in R[r] (r < 16)
// or R2[r - 16], and the LDS at lds + toff holds rows KR..m-1 only.  A
// Dijkstra step reads a register row by a wave-uniform register index (the
// row is in an SGPR), so the values and the order of the arithmetic are
// those of the all-LDS solver.  It trades VGPRs for LDS, which sets the
// number of resident LAPs when m is large.
template <int RW, int KR = 0>
__device__ void lap_solve_scalar1(double *lds, int toff, int soff, int m, double &u, double &v, int &p,
                                  double &theta, int &steps, dreg16 R = {}, dreg8 R2 = {})
{
    static_assert(KR <= 24, "at most 24 register rows");
    constexpr int KR1 = KR < 16 ? KR : 16, KR2 = KR - KR1;
    const int l = (int)(threadIdx.x & 63);
    const bool valid = l < m;
    const double *M = lds + toff;
    double *mlu = lds + soff;
    int *mlp = (int *)(mlu + m);
    int *mlw = mlp;  // the rows' proposal winners share the matching's slots: read before it is written
    const unsigned long long validm = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
    const int lc = valid ? l : 0;  // lanes past m read column 0 (never used)

    // column reduction: lane l scans column l
    constexpr int kNone = 0x7fffffff;
    u = 0.0;
    v = 0.0;
    p = -1;
    int prop = 0;
    if (valid) {
        double best;
        if constexpr (KR > 0) {
            best = R[0];
#pragma unroll
            for (int i = 1; i < KR; ++i) {
                const double x = i < 16 ? R[i] : R2[i - 16];
                if (x < best) {
                    best = x;
                    prop = i;
                }
            }
            for (int i = KR; i < m; ++i) {
                const double x = M[(i - KR) * m + l];
                if (x < best) {
                    best = x;
                    prop = i;
                }
            }
        } else {
            best = M[l];
            for (int i = 1; i < m; ++i) {
                const double x = M[i * m + l];
                if (x < best) {
                    best = x;
                    prop = i;
                }
            }
        }
        v = best;
        mlw[l] = kNone;
        mlu[l] = best;  // staged for the fold below
    }
    __builtin_amdgcn_wave_barrier();
    if (valid) atomicMin(&mlw[prop], l);
    __builtin_amdgcn_wave_barrier();
    // the LAP value starts at the left fold of the column minima
    double th = mlu[0];
    if constexpr (KR > 0) {
        // (a short unroll: a fixed m would otherwise hoist all m reads
        // while the register rows are live)
#pragma unroll 8
        for (int j = 1; j < m; ++j) th = th + mlu[j];
    } else {
        for (int j = 1; j < m; ++j) th = th + mlu[j];
    }
    __builtin_amdgcn_wave_barrier();
    int wprop = kNone, wown = kNone;
    if (valid) {
        wprop = mlw[prop];
        wown = mlw[l];
    }
    __builtin_amdgcn_wave_barrier();
    if (valid) {
        p = (wprop == l) ? prop : -1;
        mlp[l] = p;
        mlu[l] = 0.0;
    }
    unsigned long long unm = __builtin_amdgcn_ballot_w64(valid && wown == kNone);  // rows to insert
    unsigned long long freem = __builtin_amdgcn_ballot_w64(valid && p < 0);       // unmatched columns
    __builtin_amdgcn_wave_barrier();
    int st = 0;
    if (unm) {
        int i0 = (int)__builtin_ctzll(unm);
        int r = i0, last = -1;
        unsigned long long usedm = 0ull, treem = 1ull << i0;
        double minv = kInf;
        int way = -1;
        for (;;) {
            ++st;
            const unsigned long long actm = validm & ~usedm;
            const double ur = mlu[r];
            double mv;
            if (KR1 > 0 && r < KR1)
                mv = R[r];
            else if (KR2 > 0 && r < KR)
                mv = R2[r - 16];
            else {
                // the row's start as an opaque scalar, so the lane's address
                // is one add (folding KR * m into it takes a second one)
                int rb = (r - KR) * m;
                asm("" : "+s"(rb));
                mv = M[rb + lc];
            }
            const double s = (mv - ur) - v;
            const unsigned long long bm = __builtin_amdgcn_ballot_w64(s < minv) & actm;
            minv = __builtin_amdgcn_inverse_ballot_w64(bm) ? s : minv;
            way = __builtin_amdgcn_inverse_ballot_w64(bm) ? last : way;
            const double mn = part_min<RW>(minv);
            const unsigned long long eqm = __builtin_amdgcn_ballot_w64(minv == mn);
            const unsigned long long bf = eqm & freem;
            const int js = (int)__builtin_ctzll(bf != 0ull ? bf : (eqm | (1ull << 63)));
            // masked adds kept as branches over exec (one VALU op each)
            // rather than if-converted to add + two selects
            if (__builtin_amdgcn_inverse_ballot_w64(treem)) asm volatile("v_add_f64 %0, %0, %1" : "+v"(u) : "v"(mn));
            if (__builtin_amdgcn_inverse_ballot_w64(usedm)) asm volatile("v_add_f64 %0, %0, -%1" : "+v"(v) : "v"(mn));
            th = th + mn;
            const int pj = __builtin_amdgcn_readlane(p, js);
            if (pj >= 0) {
                // the search goes on: minv -= delta, and the chosen column
                // leaves it.  Its minv - mn is a zero (minv == mn there),
                // whose low word is 0, so the high word of +inf in that one
                // lane makes it exactly +inf: one select instead of two.
                // (When the search ends minv is not read.)
                minv = minv - mn;
                const int hi = __builtin_amdgcn_inverse_ballot_w64(1ull << js) ? 0x7ff00000 : __double2hiint(minv);
                minv = __hiloint2double(hi, __double2loint(minv));
                usedm |= 1ull << js;
                treem |= 1ull << pj;
                r = pj;
                last = js;
                continue;
            }
            // flip the alternating path back to the root row; the path
            // links are the lanes' own `way` registers
            if (__builtin_amdgcn_inverse_ballot_w64(treem)) mlu[l] = u;
            __builtin_amdgcn_wave_barrier();
            unsigned long long onpath = 0ull;
            int j = js;
            while (j >= 0) {
                onpath |= 1ull << j;
                j = __builtin_amdgcn_readlane(way, j);
            }
            const bool flip = __builtin_amdgcn_inverse_ballot_w64(onpath);
            int np = -1;
            if (flip) np = (way < 0) ? i0 : mlp[way];
            __builtin_amdgcn_wave_barrier();
            if (flip) {
                p = np;
                mlp[l] = np;
            }
            __builtin_amdgcn_wave_barrier();
            freem &= ~(1ull << js);
            unm &= unm - 1ull;
            if (!unm) break;
            i0 = (int)__builtin_ctzll(unm);
            r = i0;
            last = -1;
            usedm = 0ull;
            treem = 1ull << i0;
            minv = kInf;
            way = -1;
        }
    }
    theta = th;
    steps = st;
}

// Two LAPs per wavefront (m <= 32), part 0 on lanes 0-31 and part 1 on lanes
// 32-63, with the flags as wave masks (part 1 in the upper 32 bits) as in
// lap_solve_scalar1.  Each pass of the loop takes one Dijkstra step of every
// live part: the vector work (row scan, relaxation, the 32-lane minimum,
// masked updates) is shared, the choice of column, the matched row and the
// path flip are per part in scalar registers.  Part h's tile and scratch
// are at tile_off[h], scr_off[h]; nparts <= 2 parts are live.  RW = 16 when
// m <= 16: each part's live columns sit in the first 16 of its lanes and the
// minimum stops after them.
template <int RW = 32>
__device__ void lap_solve_scalar2(double *lds, const int *tile_off, const int *scr_off, int m, int nparts,
                                  double &u, double &v, int &p, double &theta, int &steps)
{
    static_assert(RW == 16 || RW == 32, "a part spans at most 32 lanes");
    const int lane = (int)(threadIdx.x & 63);
    const int h = lane >> 5;
    const int l = lane & 31;
    const bool valid = l < m && h < nparts;
    // (arithmetic, not a per-lane choice of array element: that would put
    // the two-element arrays in scratch memory)
    const int t0 = tile_off[0], t1 = tile_off[1], s0 = scr_off[0], s1 = scr_off[1];
    const double *M = lds + (t0 + h * (t1 - t0));
    double *mlu = lds + (s0 + h * (s1 - s0));
    int *mlp = (int *)(mlu + m);
    int *mlw = mlp + m;
    const unsigned long long lowm = (m >= 32) ? 0xffffffffull : ((1ull << m) - 1ull);
    const unsigned long long validm = lowm | (nparts > 1 ? (lowm << 32) : 0ull);

    // column reduction, as lap_solve_scalar1, in both parts at once
    constexpr int kNone = 0x7fffffff;
    u = 0.0;
    v = 0.0;
    p = -1;
    int prop = 0;
    if (valid) {
        double best = M[l];
        for (int i = 1; i < m; ++i) {
            const double x = M[i * m + l];
            if (x < best) {
                best = x;
                prop = i;
            }
        }
        v = best;
        mlw[l] = kNone;
        mlu[l] = best;
    }
    __builtin_amdgcn_wave_barrier();
    if (valid) atomicMin(&mlw[prop], l);
    __builtin_amdgcn_wave_barrier();
    double th = mlu[0];
    for (int j = 1; j < m; ++j) th = th + mlu[j];
    __builtin_amdgcn_wave_barrier();
    if (valid) {
        p = (mlw[prop] == l) ? prop : -1;
        mlp[l] = p;
        mlu[l] = 0.0;
    }
    const unsigned long long unm_all = __builtin_amdgcn_ballot_w64(valid && mlw[l] == kNone);
    unsigned long long freem = __builtin_amdgcn_ballot_w64(valid && p < 0);
    __builtin_amdgcn_wave_barrier();
    // per-part scalar state: rows still to insert, root row, current row,
    // last column, steps
    unsigned long long unm0 = unm_all & 0xffffffffull, unm1 = unm_all >> 32;
    bool live0 = unm0 != 0ull, live1 = unm1 != 0ull;
    int i00 = live0 ? (int)__builtin_ctzll(unm0) : 0, i01 = live1 ? (int)__builtin_ctzll(unm1) : 0;
    int r0 = i00, r1 = i01, last0 = -1, last1 = -1, st0 = 0, st1 = 0;
    unsigned long long usedm = 0ull;
    unsigned long long treem = (live0 ? 1ull << i00 : 0ull) | (live1 ? 1ull << (32 + i01) : 0ull);
    constexpr unsigned long long kUpper = 0xffffffffull << 32;  // part 1's lanes
    double minv = kInf;
    int way = -1;
    while (live0 || live1) {
        st0 += live0 ? 1 : 0;
        st1 += live1 ? 1 : 0;
        const unsigned long long livem = (live0 ? 0xffffffffull : 0ull) | (live1 ? kUpper : 0ull);
        const unsigned long long actm = validm & ~usedm & livem;
        // the lane's part picks its row: potential index and row offset are
        // formed per part in scalar registers, then selected per lane
        const int ui = __builtin_amdgcn_inverse_ballot_w64(kUpper) ? (s1 + r1) : (s0 + r0);
        const int mi = __builtin_amdgcn_inverse_ballot_w64(kUpper) ? (t1 + r1 * m) : (t0 + r0 * m);
        const double ur = lds[ui];
        const double mv = lds[mi + (l < m ? l : 0)];
        const double s = (mv - ur) - v;
        const unsigned long long bm = __builtin_amdgcn_ballot_w64(s < minv) & actm;
        minv = __builtin_amdgcn_inverse_ballot_w64(bm) ? s : minv;
        way = __builtin_amdgcn_inverse_ballot_w64(bm) ? (__builtin_amdgcn_inverse_ballot_w64(kUpper) ? last1 : last0)
                                                      : way;
        const double mn = part_min<RW>(minv);
        const unsigned long long eqm = __builtin_amdgcn_ballot_w64(minv == mn) & actm;
        const unsigned long long bf = eqm & freem;
        const unsigned f0 = (unsigned)bf, c0 = (unsigned)eqm;
        const unsigned f1 = (unsigned)(bf >> 32), c1 = (unsigned)(eqm >> 32);
        const int js0 = __builtin_ctz(f0 != 0u ? f0 : (c0 | 0x80000000u));
        const int js1 = __builtin_ctz(f1 != 0u ? f1 : (c1 | 0x80000000u));
        const unsigned long long jsm = (live0 ? 1ull << js0 : 0ull) | (live1 ? 1ull << (32 + js1) : 0ull);
        if (__builtin_amdgcn_inverse_ballot_w64(treem)) asm volatile("v_add_f64 %0, %0, %1" : "+v"(u) : "v"(mn));
        if (__builtin_amdgcn_inverse_ballot_w64(usedm)) asm volatile("v_add_f64 %0, %0, -%1" : "+v"(v) : "v"(mn));
        if (__builtin_amdgcn_inverse_ballot_w64(livem)) asm volatile("v_add_f64 %0, %0, %1" : "+v"(th) : "v"(mn));
        minv = __builtin_amdgcn_inverse_ballot_w64(jsm) ? kInf : minv - mn;
        const int pj0 = __builtin_amdgcn_readlane(p, js0);
        const int pj1 = __builtin_amdgcn_readlane(p, 32 + js1);
        const bool aug0 = live0 && pj0 < 0, aug1 = live1 && pj1 < 0;
        // a matched column extends its part's tree by its row
        if (live0 && !aug0) {
            usedm |= 1ull << js0;
            treem |= 1ull << pj0;
            r0 = pj0;
            last0 = js0;
        }
        if (live1 && !aug1) {
            usedm |= 1ull << (32 + js1);
            treem |= 1ull << (32 + pj1);
            r1 = pj1;
            last1 = js1;
        }
        if (!(aug0 || aug1)) continue;
        // an unmatched column ends its part's search: flip the alternating
        // paths of the parts that reached one (disjoint lanes, one pass)
        const unsigned long long augm = (aug0 ? 0xffffffffull : 0ull) | (aug1 ? kUpper : 0ull);
        if (__builtin_amdgcn_inverse_ballot_w64(treem & augm)) mlu[l] = u;
        __builtin_amdgcn_wave_barrier();
        unsigned long long onpath = 0ull;
        if (aug0)
            for (int j = js0; j >= 0; j = __builtin_amdgcn_readlane(way, j)) onpath |= 1ull << j;
        if (aug1)
            for (int j = js1; j >= 0; j = __builtin_amdgcn_readlane(way, 32 + j)) onpath |= 1ull << (32 + j);
        const bool flip = __builtin_amdgcn_inverse_ballot_w64(onpath);
        const int root = __builtin_amdgcn_inverse_ballot_w64(kUpper) ? i01 : i00;
        int np = -1;
        if (flip) np = (way < 0) ? root : mlp[way];
        __builtin_amdgcn_wave_barrier();
        if (flip) {
            p = np;
            mlp[l] = np;
        }
        __builtin_amdgcn_wave_barrier();
        minv = __builtin_amdgcn_inverse_ballot_w64(augm) ? kInf : minv;
        way = __builtin_amdgcn_inverse_ballot_w64(augm) ? -1 : way;
        usedm &= ~augm;
        treem &= ~augm;
        if (aug0) {
            freem &= ~(1ull << js0);
            unm0 &= unm0 - 1ull;
            live0 = unm0 != 0ull;
            if (live0) {
                i00 = (int)__builtin_ctzll(unm0);
                r0 = i00;
                last0 = -1;
                treem |= 1ull << i00;
            }
        }
        if (aug1) {
            freem &= ~(1ull << (32 + js1));
            unm1 &= unm1 - 1ull;
            live1 = unm1 != 0ull;
            if (live1) {
                i01 = (int)__builtin_ctzll(unm1);
                r1 = i01;
                last1 = -1;
                treem |= 1ull << (32 + i01);
            }
        }
    }
    theta = th;
    steps = h ? st1 : st0;
}

}  // namespace qap
