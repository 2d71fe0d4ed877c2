"""Counter-based SplitMix64 draws for cubature candidate selection (oracle).

The paper picks cubature candidates at random (Sec. 5, last paragraphs of
the cubature training).  Both implementations draw them from the same
counter-based generator, written independently from the SplitMix64
definition (Steele, Lea and Flood, OOPSLA 2014):

    fin(z):  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
             z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
    step(s) = fin(s + 0x9E3779B97F4A7C15)

Stream key for vertex i and greedy round k:
    key = step(step(step(seed) ^ i) ^ k)
draw j (j = 0, 1, ...):  u_j = step(key + j * 0x9E3779B97F4A7C15)
element index:           e_j = ((u_j >> 32) * nT) >> 32
"""
MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def _fin(z):
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def step(s):
    return _fin((s + GOLDEN) & MASK)


def stream_key(seed, i, k):
    return step(step(step(seed & MASK) ^ (i & MASK)) ^ (k & MASK))


def draw_element(key, j, nT):
    u = step((key + j * GOLDEN) & MASK)
    return ((u >> 32) * nT) >> 32


def draw_candidates(seed, i, k, nT, eligible, exclude, n_cand, max_draws_per_cand=64):
    """Up to n_cand distinct eligible elements not in ``exclude``.

    If at most n_cand such elements exist, all of them are returned in
    ascending order.  Otherwise draws are taken in order j = 0, 1, ... and an
    element is accepted if it is eligible, not excluded and not yet accepted,
    until n_cand are accepted or n_cand * max_draws_per_cand draws are spent.
    ``eligible`` is a boolean array over elements."""
    excl = set(int(e) for e in exclude)
    pool = int(eligible.sum()) - sum(1 for e in excl if eligible[e])
    if pool <= n_cand:
        return [int(e) for e in sorted(set(map(int, eligible.nonzero()[0])) - excl)]
    key = stream_key(seed, i, k)
    out, seen = [], set()
    for j in range(n_cand * max_draws_per_cand):
        e = draw_element(key, j, nT)
        if eligible[e] and e not in excl and e not in seen:
            seen.add(e)
            out.append(e)
            if len(out) == n_cand:
                break
    return out
