"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

This module holds no arithmetic of the transport method itself: it only
generates node sets, initial fields, flow parameters and the run configurations
(node counts, stencil sizes, time steps).  Both the HIP path and the CPU oracle
receive these arrays as inputs.

The paper's own node sets (icosahedral / maximum-determinant / minimum-energy
points of the SpherePts package, Section 3.1) are not available; spherical
Fibonacci points stand in for them: they are quasi-uniform with spacing
h ~ 1/sqrt(N), which is the property the method relies on.
"""
import math

import numpy as np

VEL_ZERO, VEL_SOLID, VEL_DEFORM, VEL_NL2010 = 0, 1, 2, 3
RK4, RK5F = 0, 1

# the two bell centres of the deformational-flow test (Section 4.2)
P1 = (math.sqrt(3.0) / 2.0, 0.5, 0.0)
P2 = (math.sqrt(3.0) / 2.0, -0.5, 0.0)


def fibonacci_nodes(N):
    """Spherical Fibonacci points: z_i = 1-(2i+1)/N, azimuth i * golden angle."""
    i = np.arange(N, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / N
    rho = np.sqrt((1.0 - z) * (1.0 + z))
    ga = math.pi * (3.0 - math.sqrt(5.0))
    phi = np.fmod(i * ga, 2.0 * math.pi)
    return np.ascontiguousarray(np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1))


def random_sphere_points(M, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((M, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def gaussian_bump(X, center, width):
    """exp(-|x - c|^2 / width^2)."""
    c = np.asarray(center, dtype=np.float64)
    d2 = np.sum((X - c) ** 2, axis=1)
    return np.exp(-d2 / (width * width))


def cosine_bells(X, radius=0.5):
    """0.1 + 0.9 (q1 + q2): the two C^1 cosine bells of Section 4.2."""
    q = np.zeros(X.shape[0])
    for p in (P1, P2):
        r = np.arccos(np.clip(X @ np.asarray(p), -1.0, 1.0))
        q += np.where(r < radius, 0.5 * (1.0 + np.cos(math.pi * r / radius)), 0.0)
    return 0.1 + 0.9 * q


def slotted_cylinders(X, radius=0.5, slot=1.0 / 6.0):
    """Two spherical caps of angular radius `radius` at P1, P2, each cut by a
    straight slot of width `slot` through the centre to one edge; q = 1 inside,
    0.1 elsewhere.  (Our own specification: the paper does not define it.)"""
    q = np.full(X.shape[0], 0.1)
    for p, sgn in ((P1, 1.0), (P2, -1.0)):
        p = np.asarray(p)
        r = np.arccos(np.clip(X @ p, -1.0, 1.0))
        ez = np.array([0.0, 0.0, 1.0])
        e1 = np.cross(ez, p)
        e1 /= np.linalg.norm(e1)
        a = X @ e1
        b = X @ ez
        in_cap = r < radius
        in_slot = (np.abs(a) < slot / 2.0) & (sgn * b < 0.0)
        q = np.where(in_cap & ~in_slot, 1.0, q)
    return q


def c1_bump(X):
    return np.exp(-(4.5 ** 2) * np.sum((X - np.array([1.0, 0.0, 0.0])) ** 2, axis=1))


def two_gaussians(X):
    return 0.95 * (gaussian_bump(X, P1, 0.2) + gaussian_bump(X, P2, 0.35))


def tracer_set(X, count):
    """The 8 tracer fields T0..T7 of the largest configuration (first `count`)."""
    s = 1.0 / math.sqrt(2.0)
    fields = [
        lambda: two_gaussians(X),
        lambda: gaussian_bump(X, P1, 0.2),
        lambda: gaussian_bump(X, P2, 0.35),
        lambda: gaussian_bump(X, (0.0, 0.0, 1.0), 0.2),
        lambda: gaussian_bump(X, (0.0, s, s), 0.35),
        lambda: c1_bump(X),
        lambda: cosine_bells(X),
        lambda: slotted_cylinders(X),
    ]
    return np.ascontiguousarray(np.stack([fields[i % 8]() for i in range(count)], axis=0))


def solid_body_vp(T, alpha, beta=0.0):
    """Solid-body rotation of period T about the unit axis with polar angle
    alpha and azimuth beta.  vp = [T, a0, a1, a2, 0, ...]."""
    a = (math.sin(alpha) * math.cos(beta), math.sin(alpha) * math.sin(beta), math.cos(alpha))
    return [float(T), a[0], a[1], a[2], 0.0, 0.0, 0.0, 0.0]


def tc1_vp(T=2.0 * math.pi, alpha=math.pi / 4.0):
    """Section 4.1's solid body convention: angular velocity (2pi/T)(0,-sin a,-cos a)."""
    return [float(T), 0.0, -math.sin(alpha), -math.cos(alpha), 0.0, 0.0, 0.0, 0.0]


def deform_vp(T=5.0, axis=(0.0, 0.0, 1.0), kappa=2.0):
    """Time-reversing stream-function flow: u = x x grad psi + (2pi/T) a x x,
    psi = kappa cos(pi t/T) psi0(R(t)^T x), psi0 = xyz + z^2 x / 2, R(t) the
    background rotation about a (so the flow returns exactly at t = T)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return [float(T), float(a[0]), float(a[1]), float(a[2]), float(kappa), 0.0, 0.0, 0.0]


def nl2010_vp(T=5.0):
    """The NL2010 deformational flow of Section 4.2 (rotation about e_z with
    period T; the flow reverses at T/2 and returns every parcel at T)."""
    return [float(T), 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0]


def gaussian_bells(X):
    """0.95 (exp(-5|x - p1|^2) + exp(-5|x - p2|^2)): the smooth pair of Section 4.2."""
    return 0.95 * (gaussian_bump(X, P1, 1.0 / math.sqrt(5.0)) + gaussian_bump(X, P2, 1.0 / math.sqrt(5.0)))


def paper_L(n):
    """Section 2.4: L = floor((sqrt(n) - 1)/2), i.e. the largest L with (2L+1)^2 <= n."""
    L = 0
    while (2 * (L + 1) + 1) ** 2 <= n:
        L += 1
    return L


# Run configurations.  "c2" is the headline workload.
CONFIGS = {
    "c1": dict(name="c1-solid-N1024-n31-L3-k2", N=1024, n=31, L=3, k=2, vel_id=VEL_SOLID,
               vp=tc1_vp(), dt=2.0 * math.pi / 128.0, nsteps=128, ntr=1, ic="c1_bump"),
    "c2": dict(name="c2-deform-N40962-n84-L5-k3", N=40962, n=84, L=5, k=3, vel_id=VEL_DEFORM,
               vp=deform_vp(), dt=5.0 / 480.0, nsteps=480, ntr=1, ic="two_gaussians"),
    "c3": dict(name="c3-deform-N655362-n120-L7-k4-8tr", N=655362, n=120, L=7, k=4, vel_id=VEL_DEFORM,
               vp=deform_vp(), dt=5.0 / 960.0, nsteps=960, ntr=8, ic="tracer_set"),
}


def initial_q(cfg, X):
    ic = cfg["ic"]
    if ic == "c1_bump":
        return c1_bump(X)[None, :].copy()
    if ic == "two_gaussians":
        return two_gaussians(X)[None, :].copy()
    if ic == "tracer_set":
        return tracer_set(X, cfg["ntr"])
    raise ValueError(ic)


# --------------------------------------------------------------------------
# seeded draws for the batched and served workloads
# --------------------------------------------------------------------------

class SplitMix64:
    """splitmix64 (Steele, Lea & Flood 2014); U = (x >> 11) * 2^-53."""

    def __init__(self, seed):
        self.s = seed & 0xFFFFFFFFFFFFFFFF

    def next_u64(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
        return z ^ (z >> 31)

    def uniform(self):
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def batched_runs(count=64, seed=0, nmin=2048, nmax=65536, nsteps=256,
                 pairs=((31, 3, 2), (56, 4, 2), (84, 5, 3))):
    """Independent transport runs of the batched form: N log-uniform in
    [nmin, nmax], (n, L, k) uniform over `pairs`, solid body or deformational
    flow with random axis and period, nsteps steps ending at a return time."""
    g = SplitMix64(seed)
    runs = []
    for r in range(count):
        N = int(math.floor(nmin * (nmax / nmin) ** g.uniform()))
        n, L, k = pairs[min(int(g.uniform() * len(pairs)), len(pairs) - 1)]
        deform = g.uniform() < 0.5
        alpha = math.pi * g.uniform()
        beta = 2.0 * math.pi * g.uniform()
        T = 1.0 + 9.0 * g.uniform()
        ax = (math.sin(alpha) * math.cos(beta), math.sin(alpha) * math.sin(beta), math.cos(alpha))
        if deform:
            vel_id, vp = VEL_DEFORM, deform_vp(T, ax)
        else:
            vel_id, vp = VEL_SOLID, solid_body_vp(T, alpha, beta)
        tr = min(int(g.uniform() * 8), 7)
        runs.append(dict(name=f"run{r}", N=N, n=n, L=L, k=k, vel_id=vel_id, vp=vp,
                         dt=T / nsteps, nsteps=nsteps, ntr=1, tracer=tr))
    return runs


def run_q0(run, X):
    return tracer_set(X, 8)[run["tracer"]][None, :].copy()


def served_requests(count, rate, seed=1, nmin=4096, nmax=262144, smin=64, smax=512,
                    pairs=((31, 3, 2), (56, 4, 2), (84, 5, 3), (120, 7, 4)), max_tracers=4):
    """Transport requests of the served form: Poisson arrivals at `rate` per
    second, N log-uniform in [nmin, nmax], (n, L, k) uniform over `pairs`,
    solid body or deformational flow with random axis and period, steps
    uniform in [smin, smax] (dt = T / steps, so every run ends at a return
    time), 1..max_tracers tracers drawn from the eight fields."""
    g = SplitMix64(seed)
    reqs, t = [], 0.0
    for r in range(count):
        t += -math.log(1.0 - g.uniform()) / rate
        N = int(math.floor(nmin * (nmax / nmin) ** g.uniform()))
        n, L, k = pairs[min(int(g.uniform() * len(pairs)), len(pairs) - 1)]
        deform = g.uniform() < 0.5
        alpha = math.pi * g.uniform()
        beta = 2.0 * math.pi * g.uniform()
        T = 1.0 + 9.0 * g.uniform()
        steps = smin + min(int(g.uniform() * (smax - smin + 1)), smax - smin)
        ntr = 1 + min(int(g.uniform() * max_tracers), max_tracers - 1)
        trs = [min(int(g.uniform() * 8), 7) for _ in range(ntr)]
        ax = (math.sin(alpha) * math.cos(beta), math.sin(alpha) * math.sin(beta), math.cos(alpha))
        if deform:
            vel_id, vp = VEL_DEFORM, deform_vp(T, ax)
        else:
            vel_id, vp = VEL_SOLID, solid_body_vp(T, alpha, beta)
        reqs.append(dict(name=f"req{r}", arrival=t, N=N, n=n, L=L, k=k, vel_id=vel_id, vp=vp,
                         dt=T / steps, nsteps=steps, ntr=ntr, tracers=trs))
    return reqs


def request_q0(req, X):
    fields = tracer_set(X, 8)
    return np.stack([fields[i] for i in req["tracers"]])
