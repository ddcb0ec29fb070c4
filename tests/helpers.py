"""Small test utilities: explicit ragged rows, dense views of rows, and the
sequential removal rule used as a brute-force reference."""
import numpy as np


def set_rows(P, rows, weights=None):
    """rows: list of target lists per presynaptic neuron."""
    P.len[:] = 0
    for i, tg in enumerate(rows):
        n = len(tg)
        assert n <= P.cap
        P.len[i] = n
        P.ind[i * P.cap:i * P.cap + n] = tg
        if weights is not None:
            P.w[i * P.cap:i * P.cap + n] = weights[i]


def dense(P):
    """W[post][pre] from ragged rows (fp64)."""
    W = np.zeros((P.n_post, P.n_pre))
    for i in range(P.n_pre):
        for k in range(int(P.len[i])):
            W[P.ind[i * P.cap + k], i] += P.w[i * P.cap + k]
    return W


def sequential_remove(n, remove):
    """Sequential swap-with-last removal with re-check of the moved element.
    Returns the surviving original slot ids in final slot order."""
    row = list(range(n))
    s = 0
    while s < len(row):
        if remove[row[s]]:
            row[s] = row[-1]
            row.pop()
        else:
            s += 1
    return row


def canonical_compaction(n, remove):
    """Closed-form order: holes below the new length are filled, lowest first,
    by the survivors above it taken from the highest slot down."""
    R = sum(remove)
    n2 = n - R
    holes = [s for s in range(n2) if remove[s]]
    tail = [s for s in range(n - 1, n2 - 1, -1) if not remove[s]]
    assert len(holes) == len(tail)
    row = list(range(n2))
    for h, k in zip(holes, tail):
        row[h] = k
    return row


def rows_of(P):
    out = []
    for i in range(P.n_pre):
        n = int(P.len[i])
        out.append(list(P.ind[i * P.cap:i * P.cap + n]))
    return out


def bits_to_sets(bits, n_pre, n_post):
    words = (n_post + 31) // 32
    b = bits.reshape(n_pre, words)
    out = []
    for i in range(n_pre):
        s = set()
        for j in range(n_post):
            if (int(b[i, j >> 5]) >> (j & 31)) & 1:
                s.add(j)
        out.append(s)
    return out


def numpy_block(key0, key1, ctr):
    # numpy advances the counter before producing a block, so the block at
    # counter c is the first output of a generator started at c - 1.
    c = np.array(ctr, dtype=np.uint64)
    c0 = [int(x) for x in c]
    # subtract one with borrow over the 256-bit counter
    for k in range(4):
        if c0[k] > 0:
            c0[k] -= 1
            break
        c0[k] = (1 << 64) - 1
    bg = np.random.Philox(key=np.array([key0, key1], dtype=np.uint64),
                          counter=np.array(c0, dtype=np.uint64))
    return np.array(bg.random_raw(4), dtype=np.uint64)
