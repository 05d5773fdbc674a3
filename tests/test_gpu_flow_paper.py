"""The paper's two flow checks (Sec. 4.2) on the GPU.

Double-Poiseuille viscosity (the Backer et al. set-up): no conservative
force, density 6, k_B T = 0.5, sigma = 4.5 (so gamma = sigma^2 / (2 k_B T)
= 20.25 by Eq (9)), the standard weight w_R = 1 - r/r_c (s = 1), dt =
0.001, 4,608 particles in 12 x 8 x 8 with a body force 0.055 along the
8-long axis whose sign flips between the two halves of the 12-long axis;
10 replicas with their own configurations and random streams.  Each
replica's binned start-up profiles over t <= 60 are fitted with Eq (10) for
the kinematic viscosity nu; the dynamic viscosity rho nu is the figure the
paper reports (2.089 +- 0.009, against 2.09 +- 0.02 published).

Transient double Poiseuille: density 5, a = 15, sigma = 3, k_B T = 1,
dt = 0.01, s = 1, 262,144 particles in 59.4123 x 7.42654 x 118.825, the
flow along the first axis and its sign flipping between the halves of the
118.825-long axis; velocity profiles over the windows [T - 0.5, T + 0.5] at
T = 100, 200, 500 and 1000.  The paper does not state the body force; F =
0.001 keeps the peak velocity near 1 (well below the fluid's sound speed).
One viscosity fits all four windows with Eq (10).

The library drives the body force along x with its sign flipping at half
the y extent, so each box is given with the paper's axes permuted (flow ->
x, gradient -> y)."""
import numpy as np
import pytest

import dpd_inputs as di

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]
P = pytest.importorskip("paper_1311_0402_amd")
scipy_opt = pytest.importorskip("scipy.optimize")


def _eq10(z, t, nu, g, d, modes=60):
    """Eq (10): start-up velocity of a channel of width d under body force
    g, z measured from the channel centre."""
    u = g / (2 * nu) * (d * d / 4 - z * z)
    for n in range(modes):
        k = 2 * n + 1
        u = u - ((-1) ** n * 4 * g * d * d / (nu * np.pi ** 3 * k ** 3)
                 * np.cos(k * np.pi * z / d) * np.exp(-k * k * np.pi ** 2 * nu * t / (d * d)))
    return u


def _fit_nu(prof, times, ly, g, nb, bounds):
    """Least-squares nu over all windows and both channels (the upper one
    flows the other way); returns nu and the RMS residual."""
    y = (np.arange(nb) + 0.5) * ly / nb
    d = ly / 2
    chans = []
    for lo, sign in ((0.0, 1.0), (d, -1.0)):
        m = (y > lo) & (y < lo + d)
        chans.append((m, y[m] - (lo + d / 2), sign))

    def resid(nu):
        out = []
        for w, ts in enumerate(times):
            for m, z, sign in chans:
                mod = np.mean([_eq10(z, t, nu, g, d) for t in ts], axis=0)
                out.append(sign * prof[w][m] - mod)
        return np.concatenate(out)

    r = scipy_opt.minimize_scalar(lambda nu: np.sum(resid(nu) ** 2), bounds=bounds, method="bounded")
    return float(r.x), float(np.sqrt(np.mean(resid(float(r.x)) ** 2)))


def test_backer_double_poiseuille_viscosity():
    kbt, rho, g, dt = 0.5, 6.0, 0.055, 0.001
    sigma = 4.5
    gamma = sigma * sigma / (2 * kbt)
    box = (8.0, 12.0, 8.0)
    reps, nb, every, window, t_end = 10, 24, 50, 5000, 60.0
    n = int(round(rho * np.prod(box)))
    assert n == 4608
    systems = []
    for r in range(reps):
        s = di.uniform_fluid(n, box, 100 + r, a=0.0, gamma=gamma, sigma=sigma, s=1.0, dt=dt, kbt=kbt)
        s.body_g, s.body_split = g, 0.5 * box[1]
        s.seed = di.splitmix64(1000 + r)
        systems.append(s)
    bt = P.Batch([P.Params.like(s) for s in systems], [n] * reps, P.FP64)
    bt.load(np.concatenate([s.x for s in systems], 1), np.concatenate([s.v for s in systems], 1),
            np.concatenate([s.tag for s in systems]), np.concatenate([s.type for s in systems]))
    steps = int(round(t_end / dt))
    n_win = steps // window
    prof = torch.zeros((n_win, reps * nb), dtype=torch.float64, device="cuda")
    cnt = torch.zeros_like(prof)
    sid = torch.repeat_interleave(torch.arange(reps, device="cuda"), n)
    times = [[] for _ in range(n_win)]
    kt = []
    for k in range(steps // every):
        bt.step(every)
        step = (k + 1) * every
        w = (step - 1) // window
        st = bt.state
        b = torch.clamp((st.x[1] * (nb / box[1])).long(), 0, nb - 1) + sid * nb
        prof[w].index_add_(0, b, st.v[0])
        cnt[w].index_add_(0, b, torch.ones_like(st.v[0]))
        times[w].append(step * dt)
        if step > steps // 2:
            kt.append((st.v[1:] ** 2).sum() / (2 * reps * n))
    torch.cuda.synchronize()
    bt.check_status()
    prof = (prof / cnt).cpu().numpy().reshape(n_win, reps, nb)
    nus = np.array([_fit_nu(prof[:, r], [ts[::4] for ts in times], box[1], g, nb, (0.02, 5.0))[0]
                    for r in range(reps)])
    eta, eta_err = rho * nus.mean(), rho * nus.std(ddof=1) / np.sqrt(reps)
    kbt_meas = float(torch.stack(kt).mean().item())
    print(f"dynamic viscosity {eta:.4f} +- {eta_err:.4f} (paper 2.089 +- 0.009; published 2.09 +- 0.02), "
          f"k_BT {kbt_meas:.4f}", flush=True)
    # the paper's value within three combined standard errors
    assert abs(eta - 2.089) <= 3.0 * np.hypot(eta_err, 0.009), (eta, eta_err)
    assert eta_err < 0.02
    assert abs(kbt_meas - kbt) < 0.01 * kbt, kbt_meas


def test_transient_double_poiseuille_follows_eq10():
    rho, g, dt = 5.0, 0.001, 0.01
    box = (59.4123, 118.825, 7.42654)       # the paper's (x, z, y)
    n = 262_144
    assert abs(n / np.prod(box) - rho) < 1e-4
    s = di.uniform_fluid(n, box, 77, a=15.0, gamma=4.5, sigma=3.0, s=1.0, dt=dt)
    s.body_g, s.body_split = g, 0.5 * box[1]
    sim = P.System(P.Params.like(s), n, P.FP64)
    sim.load(s.x, s.v, s.tag, s.type)
    nb, every = 60, 10
    prof, times = [], []
    done = 0
    for T in (100, 200, 500, 1000):
        start = int(round((T - 0.5) / dt))
        if start > done:
            sim.step(start - done)
            done = start
        acc = torch.zeros(nb, dtype=torch.float64, device="cuda")
        cnt = torch.zeros(nb, dtype=torch.float64, device="cuda")
        ts = []
        for _ in range(int(round(1.0 / dt)) // every):
            sim.step(every)
            done += every
            st = sim.state
            b = torch.clamp((st.x[1] * (nb / box[1])).long(), 0, nb - 1)
            acc.index_add_(0, b, st.v[0])
            cnt.index_add_(0, b, torch.ones_like(st.v[0]))
            ts.append(done * dt)
        prof.append((acc / cnt).cpu().numpy())
        times.append(ts)
        print(f"T = {T}: peak {np.abs(prof[-1]).max():.3f}", flush=True)
    torch.cuda.synchronize()
    sim.check_status()
    nu, rms = _fit_nu(prof, times, box[1], g, nb, (0.05, 5.0))
    peak = g * (box[1] / 2) ** 2 / (8 * nu)
    print(f"transient fit: nu {nu:.4f}, rms residual {rms:.4f} (steady peak {peak:.3f})", flush=True)
    assert 0.1 < nu < 2.0, nu
    # one viscosity describes all four windows within the bins' noise
    assert rms < 0.03 * peak, (rms, peak)
