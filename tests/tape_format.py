"""Conversions between the oracle's step tape order (type, order, value,
then for a step the n_species state values) and the library's entry format
([type, state of a step, order, value, type]), so that tapes written by
either side can be walked by the other."""
import numpy as np

SCALARS = 4  # doubles of a library tape entry besides the state


def to_device(vals, N):
    """An oracle tape in the library's entry format."""
    out, p = [], 0
    while p < len(vals):
        typ, order, x = vals[p:p + 3]
        n = N if int(typ) == 2 else 0
        out.append(typ)
        out.extend(vals[p + 3:p + 3 + n])
        out.extend([order, x, typ])
        p += 3 + n
    return np.array(out)


def to_oracle(dev_vals, N):
    """A library tape back in the oracle's order (parsed from the start)."""
    entries, p = [], 0
    while p < len(dev_vals):
        typ = dev_vals[p]
        n = N if int(typ) == 2 else 0
        order, x, typ2 = dev_vals[p + 1 + n:p + 4 + n]
        assert typ2 == typ, "malformed tape"
        entries.append(np.concatenate([[typ, order, x], dev_vals[p + 1:p + 1 + n]]))
        p += SCALARS + n
    return np.concatenate(entries) if entries else np.zeros(0)


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


def entry_offsets(dev_vals, N):
    """Start offsets of the entries of a library tape."""
    out, p = [], 0
    while p < len(dev_vals):
        out.append(p)
        p += SCALARS + (N if int(dev_vals[p]) == 2 else 0)
    return out
