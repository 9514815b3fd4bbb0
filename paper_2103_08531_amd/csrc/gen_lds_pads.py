"""Writes vgf_lds_pads.hpp: the LDS pad of each exchange of a line held by
one wavefront (the multiply passes along the contiguous axis).

A line of P points that stage e writes and stage e+1 reads sits in LDS at
position p + k (p >> s) (a pad of k slots every 2^s positions; line l of the
wavefront's tile starts at l * LP, LP = P + P/8). For every FFT length,
direction, exchange and lanes-per-line count the kernels use, this script
picks (k, s) by counting bank conflicts under the measured model of 8-byte
LDS accesses: a write is resolved per 32 lanes over 32 slots of 8 bytes
(slot = index mod 32), a read per 16 lanes over 16 slots (index mod 16); an
access takes one extra cycle per lane beyond the first on its busiest slot.
Other pads must keep every access additive in the butterfly input r (one
per-lane base plus r times a constant) and within LP; the pad of one slot
every 8 positions (addressed per access where it is not additive) is kept
unless another pad has strictly fewer extra cycles.

Run: python3 gen_lds_pads.py > vgf_lds_pads.hpp
"""
import sys

LENGTHS = [16, 24, 32, 36, 48, 64, 72, 96, 108, 128, 144, 192, 216, 256, 288, 324, 384, 432,
           512, 576, 648, 768, 864, 972, 1024, 1152, 1296, 1536, 1728, 1944, 2048]


def pow2(P):
    return (P & -P).bit_length() - 1


def pow3(P):
    x, b = P >> pow2(P), 0
    while x % 3 == 0:
        x //= 3
        b += 1
    return b


def radix6_plan(P):
    return pow2(P) % 3 == 1 and pow2(P) >= 4 and pow3(P) >= 1 and (P // 6 <= 64 or (P // 6) % 64 == 0)


def fwd_radix(P, s):
    a = pow2(P)
    q, r = a // 3, a % 3
    if radix6_plan(P):
        return 8 if s < q else (6 if s == q else 3)
    s2 = q + (1 if r else 0)
    if s >= s2:
        return 3
    if r == 0:
        return 8
    if r == 2:
        return 8 if s < q else 4
    if q == 0:
        return 2
    return 8 if s < q - 1 else 4


def radices(P, sign):
    a = pow2(P)
    n = (a // 3 if radix6_plan(P) else a // 3 + (1 if a % 3 else 0)) + pow3(P)
    f = [fwd_radix(P, s) for s in range(n)]
    return f if sign < 0 else f[::-1]


def wave_nq(P):
    nq = 1
    while nq * 8 < P and nq * 2 <= 64:
        nq *= 2
    return nq


def rows(P, rad, nq, s, kind):
    """For each (task, r): the 64 lanes' (position, line) or None."""
    R = rad[s]
    NB = P // R
    NS = 1
    for k in range(s):
        NS *= rad[k]
    out = []
    for t in range((NB + nq - 1) // nq):
        for r in range(R):
            row = []
            for lane in range(64):
                l, q = lane // nq, lane % nq
                j = q + t * nq
                if l >= 64 // nq or j >= NB:
                    row.append(None)
                    continue
                pos = j + r * NB if kind == "in" else (j // NS) * NS * R + (j % NS) + r * NS
                row.append((pos, l, j, r, t))
            out.append(row)
    return out


def extra_cycles(addrs, group, mod):
    c = 0
    for g0 in range(0, 64, group):
        cnt = {}
        for a in addrs[g0:g0 + group]:
            if a is not None:
                cnt[a % mod] = cnt.get(a % mod, 0) + 1
        if cnt:
            c += max(cnt.values()) - 1
    return c


def evaluate(P, rad, nq, e, k, s, additive=True):
    LP = P + P // 8
    f = lambda p: p + k * (p >> s)
    if f(P - 1) >= LP:
        return None
    cost = 0
    for kind, st, group, mod in (("out", e, 32, 32), ("in", e + 1, 16, 16)):
        rr = rows(P, rad, nq, st, kind)
        # additivity in r: f(pos(j, r)) - f(pos(j, 0)) == r * step for every lane
        R = rad[st]
        NB = P // R
        NS = 1
        for x in range(st):
            NS *= rad[x]
        p0 = lambda j: j if kind == "in" else (j // NS) * NS * R + (j % NS)
        step = f(p0(0) + (NB if kind == "in" else NS)) - f(p0(0))
        for row in rr:
            for a in row:
                if a is None or not additive:
                    continue
                pos, l, j, r, t = a
                if f(pos) - f(p0(j)) != r * step:
                    return None
        for row in rr:
            cost += extra_cycles([None if a is None else a[1] * LP + f(a[0]) for a in row], group, mod)
    return cost


def best_pad(P, sign, e, nq):
    rad = radices(P, sign)
    # the kernels address the pad of one slot every 8 per access where it is
    # not additive, so it is compared without that condition
    base = evaluate(P, rad, nq, e, 1, 3, additive=False)
    best = (base, 1, 3)
    for s in range(2, 12):
        for k in range(0, 17):
            c = evaluate(P, rad, nq, e, k, s)
            if c is not None and c < best[0]:
                best = (c, k, s)
    return best, base


def main():
    entries = []
    for P in LENGTHS:
        nq0 = wave_nq(P)
        for nq in sorted({nq0, max(1, nq0 // 2)}):
            for sign in (-1, 1):
                rad = radices(P, sign)
                for e in range(len(rad) - 1):
                    (c, k, s), base = best_pad(P, sign, e, nq)
                    entries.append((P, sign, e, nq, k, s, c, base))
    w = sys.stdout.write
    w("// Generated by gen_lds_pads.py (do not edit): LDS pad per exchange of a\n")
    w("// line held by one wavefront. Entry {P, sign, exchange, lanes per line,\n")
    w("// k, s}: the line's position p sits at p + k * (p >> s). Extra cycles per\n")
    w("// exchange under the bank model (this pad / one slot every 8): see each line.\n")
    w("#pragma once\n\nnamespace vgf {\n\nstruct LdsPad {\n  int P, sign, e, nq, k, s;\n};\n\n")
    w("constexpr LdsPad kLdsPads[] = {\n")
    for (P, sign, e, nq, k, s, c, base) in entries:
        w("    {%d, %d, %d, %d, %d, %d},  // %d / %s\n" % (P, sign, e, nq, k, s, c, base))
    w("};\n\n")
    w("// (k, s) of exchange e (stage e writes, stage e + 1 reads) of a length-P\n")
    w("// transform in direction sign with nq lanes per line; one slot every 8\n")
    w("// positions where the table has no entry.\n")
    w("constexpr LdsPad lds_pad(int P, int sign, int e, int nq) {\n")
    w("  for (const LdsPad& p : kLdsPads)\n")
    w("    if (p.P == P && p.sign == sign && p.e == e && p.nq == nq) return p;\n")
    w("  return LdsPad{P, sign, e, nq, 1, 3};\n}\n\n}  // namespace vgf\n")


if __name__ == "__main__":
    main()
