"""A second, independent writing of the filter in plain Python (strings and
sets), used only to cross-check the C oracle.  Written from the method
statement (Sec. 2.1, Sec. 3.3, Sec. 3.4) with the same readings, but with
different idioms: masks are sets of mismatch positions, amendment is a scan
for gaps between consecutive mismatches."""

CODE = {"A": 0, "C": 1, "G": 2, "T": 3}


def mismatches(read, window, d):
    """Positions i where read[i-d] (or 'A' outside the read) differs from window[i]."""
    m = len(read)
    out = set()
    for i in range(m):
        j = i - d
        rb = CODE[read[j]] if 0 <= j < m else 0
        x = rb ^ CODE[window[i]]
        if x & 1 or x & 2:
            out.add(i)
    return out


def amended(ones, m):
    """Fill every gap of 1 or 2 positions between two consecutive 1s."""
    pts = sorted(ones)
    out = set(pts)
    for a, b in zip(pts, pts[1:]):
        if 2 <= b - a <= 3:
            out.update(range(a + 1, b))
    return out


def gatekeeper_gpu(read, window, e, refine=True):
    read, window = read.upper(), window.upper()
    m = len(read)
    if m == 0 or m > 512:
        return 3, 0xFFFF
    if len(window) < m or any(c not in CODE for c in read + window[:m]):
        return 2, 0xFFFF
    window = window[:m]
    final = set(range(m))
    for k in range(0, min(e, m) + 1):
        for d in ((0,) if k == 0 else (k, -k)):
            mask = amended(mismatches(read, window, d), m)
            if refine and d > 0:
                mask |= set(range(0, min(d, m)))
            if refine and d < 0:
                mask |= set(range(max(0, m + d), m))
            final &= mask
    est = len(final)
    return (1 if est <= e else 0), est
