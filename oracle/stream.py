"""Overlap-save segmentation of a long strain (test infrastructure only; see
package docstring).

Reading (Sec. III.E and the cost estimate of Sec. III.F): the data are cut
into segments of N samples, each overlapping the previous one by N/2, so a
segment contributes N/2 unique SNR samples.  Segment i starts at i N/2 (the
last one at n - N when n - N is not a multiple of N/2); its valid samples are
the central half [start + N/4, start + 3N/4), except that the first segment's
window starts at 0 and the last one's ends at n, and where the last segment
was moved back its window starts where the previous one ended.  The windows
partition [0, n): every sample of the stream is reported by exactly one
segment.
"""
from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np

from . import mf


def segments(n: int, N: int) -> List[Tuple[int, int, int]]:
    """(start, lo, hi) of every segment: the segment is strain[start:start+N]
    and reports the stream samples lo <= m < hi."""
    if n < N or N % 4:
        raise ValueError("need n >= N and N divisible by 4")
    hop = N // 2
    count = -(-(n - N) // hop) + 1
    starts = [min(i * hop, n - N) for i in range(count)]
    out = []
    for i, s in enumerate(starts):
        lo = 0 if i == 0 else out[-1][2]
        hi = n if i == count - 1 else starts[i + 1] + N // 4
        out.append((s, lo, hi))
    return out


def stream_triggers(strain: np.ndarray, N: int, search: Callable[[np.ndarray], np.ndarray]) -> np.ndarray:
    """Triggers of a long strain: `search(segment)` returns a TRIGGER_DTYPE
    array with segment-relative samples; the windowed triggers of each
    segment, shifted to stream samples, are concatenated in segment order
    (within a segment the order of `search`)."""
    parts = []
    for s, lo, hi in segments(strain.shape[0], N):
        t = search(strain[s:s + N]).copy()
        t["sample"] += s
        parts.append(t[(t["sample"] >= lo) & (t["sample"] < hi)])
    if not parts:
        return np.empty(0, dtype=mf.TRIGGER_DTYPE)
    return np.concatenate(parts)
