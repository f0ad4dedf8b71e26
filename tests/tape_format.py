"""Conversions between the oracle's step tape order (type, order, value,
then for a step the n_species state values) and the reverse-mode kernel's
entry format (the state first, then order, value, type), so that tapes
written by either side can be walked by the other."""
import numpy as np


def to_device(vals, N):
    """An oracle tape in the reverse-mode entry format."""
    out, p = [], 0
    while p < len(vals):
        typ, order, x = vals[p:p + 3]
        n = N if int(typ) == 2 else 0
        out.extend(vals[p + 3:p + 3 + n])
        out.extend([order, x, typ])
        p += 3 + n
    return np.array(out)


def to_oracle(dev_vals, N):
    """A tape in the reverse-mode entry format back in the oracle's order
    (parsed from the end, as the kernel walks it)."""
    entries, p = [], len(dev_vals)
    while p > 0:
        typ, x, order = dev_vals[p - 1], dev_vals[p - 2], dev_vals[p - 3]
        n = N if int(typ) == 2 else 0
        entries.append(np.concatenate([[typ, order, x], dev_vals[p - 3 - n:p - 3]]))
        p -= 3 + n
    return np.concatenate(entries[::-1]) if entries else np.zeros(0)


def pack(tapes, pad=5):
    """Per-cell tapes as one [n_cells][stride] buffer (NaN beyond each
    tape's end) and their lengths."""
    stride = max(len(t) for t in tapes) + pad
    buf = np.full((len(tapes), stride), np.nan)
    for i, t in enumerate(tapes):
        buf[i, :len(t)] = t
    return buf, np.array([len(t) for t in tapes], dtype=np.int64)


def count_steps(vals, N):
    """Accepted steps on an oracle-order tape."""
    p, n = 0, 0
    while p < len(vals):
        n += int(vals[p]) == 2
        p += 3 + (N if int(vals[p]) == 2 else 0)
    return n
