"""Hand-built tiny networks for closed-form tests."""
import numpy as np


def hand_net(n, edges, is_inh=None, region=None, n_regions=1, max_delay=5, V0=None,
             g=(0.023125, 0.00115625, 0.32, 0.008), Iext=0.0, bg_lambda=0.0, bg_w=0.41686201,
             seed=3, tau_ms=(2.0, 40.0, 10.0, 50.0), dt_ms=1.0, tref_ms=2.0, member=0):
    """Build a Network by hand from a list of (post, pre, delay, weight)."""
    from netgen import Network
    edges = sorted(edges, key=lambda e: (e[0], e[1], e[2]))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    for e in edges:
        row_ptr[e[0] + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    col = np.array([e[1] for e in edges], dtype=np.int32)
    delay = np.array([e[2] for e in edges], dtype=np.uint8)
    w = np.array([e[3] for e in edges], dtype=np.float32)
    region = np.zeros(n, dtype=np.int32) if region is None else np.asarray(region, dtype=np.int32)
    is_inh = np.zeros(n, dtype=np.uint8) if is_inh is None else np.asarray(is_inh, dtype=np.uint8)
    V0 = np.full(n, -65.0, dtype=np.float32) if V0 is None else np.asarray(V0, dtype=np.float32)
    ptypes = np.array([[1.0, 0.03, -75.0, -50.0, -65.0, tref_ms, Iext, *g]], dtype=np.float32)
    return Network(n=n, n_regions=n_regions, max_delay=max_delay, row_ptr=row_ptr, col=col, w=w,
                   delay=delay, is_inh=is_inh, region=region, ptype=np.zeros(n, dtype=np.uint16),
                   ptypes=ptypes, V0=V0, E=np.array([0.0, 0.0, -70.0, -100.0], dtype=np.float32),
                   tau_ms=np.array(tau_ms, dtype=np.float32), dt_ms=float(dt_ms),
                   bg_lambda=float(bg_lambda), bg_w=float(np.float32(bg_w)), seed=int(seed),
                   member=int(member), name="hand_net")
