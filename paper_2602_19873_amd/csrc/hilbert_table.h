// Hilbert keys (Sec. II-A: Hilbert order) by a level state machine.
//
// The transpose algorithm of hilbert_key (sort.hip) walks the 21 levels from
// the top. When it reaches a level, the operations of the levels above have
// applied a signed permutation of the three axes to that level's bits (a
// level inverts axis 0 or exchanges it with axis i, both on every lower
// bit), and the flip that follows the Gray step is the parity of the
// Gray-coded axis-2 bits above the level. So (axis permutation, inversions,
// parity) is a state, and one level maps (state, the level's three
// coordinate bits) to (its 3-bit key digit, the next state). Of the 96
// states 48 are reachable from the start. The tables below are built at
// compile time from that description: one for the top level (20) from the
// start state, and one that takes two levels per lookup, so a key costs 11
// lookups instead of 20 levels of data-dependent selects.
#pragma once

#include <stdint.h>

namespace sfcnl {
namespace hilbert {

constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
constexpr int kStates = 48;  // reachable states

constexpr int perm_index(int p0, int p1, int p2) {
    for (int i = 0; i < 6; i++)
        if (kPerm[i][0] == p0 && kPerm[i][1] == p1 && kPerm[i][2] == p2) return i;
    return -1;
}

// Full state numbering: perm * 16 + inversions * 2 + parity. One level:
// bits c_i = o[perm[i]] ^ inv_i (o: axis 0 in bit 2 of oct); the digit is the
// Gray code of c with the parity flip; the next state applies the level's
// operations (for i = 0, 1, 2: c_i set inverts axis 0, else axis 0 and axis
// i exchange places) and adds the level's Gray-coded axis-2 bit to the parity.
struct Step {
    int digit, next;
};
constexpr Step step(int st, int oct) {
    int p[3] = {kPerm[st >> 4][0], kPerm[st >> 4][1], kPerm[st >> 4][2]};
    int s[3] = {(st >> 1) & 1, (st >> 2) & 1, (st >> 3) & 1};
    const int par = st & 1;
    const int o[3] = {(oct >> 2) & 1, (oct >> 1) & 1, oct & 1};
    int c[3] = {0, 0, 0};
    for (int i = 0; i < 3; i++) c[i] = o[p[i]] ^ s[i];
    const int g0 = c[0], g1 = c[1] ^ c[0], g2 = c[2] ^ c[1] ^ c[0];
    for (int i = 0; i < 3; i++) {
        if (c[i]) {
            s[0] ^= 1;
        } else if (i != 0) {
            const int tp = p[0], ts = s[0];
            p[0] = p[i];
            s[0] = s[i];
            p[i] = tp;
            s[i] = ts;
        }
    }
    return Step{((g0 ^ par) << 2) | ((g1 ^ par) << 1) | (g2 ^ par),
                perm_index(p[0], p[1], p[2]) * 16 + ((s[0] | (s[1] << 1) | (s[2] << 2)) << 1) + (par ^ g2)};
}

// start[oct]: level 20 from the start state, entry next << 3 | digit.
// pair[st << 6 | x2 << 4 | y2 << 2 | z2] with x2 = the axis-0 bits of levels
// (k + 1, k) (level k + 1 the high bit), likewise y2, z2: entry next << 6 |
// digit(k + 1) << 3 | digit(k). States are numbered densely over the
// reachable ones.
struct Tables {
    uint16_t start[8];
    uint16_t pair[kStates * 64];
};

constexpr Tables build() {
    int dense[96] = {};
    for (int i = 0; i < 96; i++) dense[i] = -1;
    int order[96] = {};
    int n = 0;
    dense[0] = n;
    order[n++] = 0;
    for (int q = 0; q < n; q++)
        for (int oct = 0; oct < 8; oct++) {
            const int nx = step(order[q], oct).next;
            if (dense[nx] < 0) {
                dense[nx] = n;
                order[n++] = nx;
            }
        }
    Tables t = {};
    for (int oct = 0; oct < 8; oct++) {
        const Step a = step(0, oct);
        t.start[oct] = (uint16_t)(dense[a.next] << 3 | a.digit);
    }
    for (int d = 0; d < n && d < kStates; d++)
        for (int idx = 0; idx < 64; idx++) {
            const int x2 = idx >> 4, y2 = (idx >> 2) & 3, z2 = idx & 3;
            const int hi = ((x2 >> 1) << 2) | ((y2 >> 1) << 1) | (z2 >> 1);
            const int lo = ((x2 & 1) << 2) | ((y2 & 1) << 1) | (z2 & 1);
            const Step a = step(order[d], hi);
            const Step b = step(a.next, lo);
            t.pair[d * 64 + idx] = (uint16_t)(dense[b.next] << 6 | a.digit << 3 | b.digit);
        }
    return t;
}

constexpr Tables kTables = build();
static_assert(kTables.pair[0] != 0xFFFF, "table built");

}  // namespace hilbert
}  // namespace sfcnl
