"""Philox4x64-10 counter-based generator, written out in plain Python integers.

Test infrastructure only (see ``oracle/__init__.py``).

Definition followed: Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11), the Philox-4x64 bijection with 10 rounds.  One
round maps the counter (x0, x1, x2, x3) under the round key (k0, k1) to

    y0 = hi(M1*x2) ^ x1 ^ k0,  y1 = lo(M1*x2),
    y2 = hi(M0*x0) ^ x3 ^ k1,  y3 = lo(M0*x0),

where hi/lo are the upper/lower 64 bits of the 128-bit product, and the key
is bumped by the Weyl constants (W0, W1) between rounds.

How the CP method consumes the stream (the paper only says "Randsample" and
"uniformly sample n", Algorithms 2-5; this mapping is our reading):
key = (seed, stream_id); step t, draw d uses counter (t, d // 4, 0, 0) and
output word d % 4.  Draw 0 is the mode draw, draw 1 + s*B + f is fibre f of
the s-th sampled mode (modes k != n in ascending order).
"""

MASK64 = (1 << 64) - 1

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B

ROUNDS = 10


def philox4x64(counter, key, rounds=ROUNDS):
    """Apply the Philox-4x64 bijection to a 4-word counter under a 2-word key."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = (
            ((p1 >> 64) ^ x1 ^ k0) & MASK64,
            p1 & MASK64,
            ((p0 >> 64) ^ x3 ^ k1) & MASK64,
            p0 & MASK64,
        )
    return (x0, x1, x2, x3)


def draw_word(seed, stream_id, t, d):
    """64-bit uniform word for draw ``d`` of step ``t`` (layout in module doc)."""
    block = philox4x64((t, d // 4, 0, 0), (seed, stream_id))
    return block[d % 4]


def draw_words(seed, stream_id, t, count):
    """Words for draws 0..count-1 of step ``t`` (one Philox call per 4 draws)."""
    out = []
    for blk in range((count + 3) // 4):
        out.extend(philox4x64((t, blk, 0, 0), (seed, stream_id)))
    return out[:count]


def mulhi64(u, n):
    """floor(u * n / 2**64) for a 64-bit word u and a non-negative integer n."""
    return (int(u) * int(n)) >> 64
