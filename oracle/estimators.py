"""Power-spectrum and FFT-bispectrum estimators (FP64).

Test infrastructure only (see ``oracle/__init__``).

Definitions: eq. powerspectrum, <delta(k1) delta(k2)> = (2 pi)^3 delta_D(k1+k2) P(k1),
and eq. bispectre, <delta(k1) delta(k2) delta(k3)> = (2 pi)^3 delta_D(k1+k2+k3) B.
With the continuum amplitude (V/N^3) dhat and (2 pi)^3 delta_D(0) = V,

    P = (V / N^6) <|dhat|^2>_shell,     B = (V^2 / N^9) <dhat dhat dhat>_closed triangles.

Power-spectrum bins (binning is not stated in the paper; reading): bin width
w = (N/2)/n_bins in units of k_f, bin b holds the modes with
w (b + 1/2) <= |n| < w (b + 3/2), decided in integers as
N^2 (2b+1)^2 <= 16 n_bins^2 |n|^2 < N^2 (2b+3)^2.  k = 0 and corner modes beyond
the last bin are dropped.  The raw estimator is returned: no shot-noise
subtraction and no CIC deconvolution.

Bispectrum (FFT shell estimator): for shells S_i with centre c_i and width w
(units of k_f; membership (2c - w)^2 <= 4|n|^2 < (2c + w)^2 evaluated in
float64), delta_i = IDFT(dhat 1_{S_i}) and I_i = IDFT(1_{S_i}); then
    sum_x delta_a delta_b delta_c = N^-6 sum_{n1+n2+n3=0} dhat dhat dhat,
    sum_x I_a I_b I_c             = N^-6 N_tri,
so B = (V^2/N^9) sum_x delta_a delta_b delta_c / sum_x I_a I_b I_c.  The paper's
squeezed configurations fix k3 = 4 k_f (Sec. 4.2).
"""
from __future__ import annotations

import math

import torch

from . import fourier


def mode_norm_sq(n: int) -> torch.Tensor:
    """|n|^2 (integer) on the r2c grid, int64 [N,N,N/2+1]."""
    nx, ny, nz = fourier.int_freqs(n)
    return (nx * nx + ny * ny + nz * nz).expand(n, n, n // 2 + 1)


def pk_bin_index(n: int, n_bins: int) -> torch.Tensor:
    """Bin of each r2c mode (-1 if in no bin), decided in integers."""
    s = 16 * n_bins * n_bins * mode_norm_sq(n)
    out = torch.full(s.shape, -1, dtype=torch.long)
    for b in range(n_bins):
        lo = n * n * (2 * b + 1) ** 2
        hi = n * n * (2 * b + 3) ** 2
        out = torch.where((s >= lo) & (s < hi), torch.full_like(out, b), out)
    return out


def power_spectrum_from_k(dhat: torch.Tensor, n: int, box: float, n_bins: int):
    """(k_mean [h/Mpc], P [(Mpc/h)^3], n_modes) from r2c amplitudes."""
    b = pk_bin_index(n, n_bins).reshape(-1)
    wt = fourier.r2c_weights(n).expand(n, n, n // 2 + 1).reshape(-1)
    p2 = (dhat.real ** 2 + dhat.imag ** 2).reshape(-1)
    kmag = torch.sqrt(mode_norm_sq(n).double()).reshape(-1)
    sel = b >= 0
    cnt = torch.zeros(n_bins, dtype=torch.float64).index_add(0, b[sel], wt[sel])
    sp = torch.zeros(n_bins, dtype=torch.float64).index_add(0, b[sel], (wt * p2)[sel])
    sk = torch.zeros(n_bins, dtype=torch.float64).index_add(0, b[sel], (wt * kmag)[sel])
    kf = 2.0 * math.pi / box
    vol = box ** 3
    safe = torch.where(cnt > 0, cnt, torch.ones_like(cnt))
    pk = torch.where(cnt > 0, vol / n ** 6 * sp / safe, torch.zeros_like(cnt))
    km = torch.where(cnt > 0, kf * sk / safe, torch.zeros_like(cnt))
    return km, pk, cnt.round().long()


def power_spectrum(delta: torch.Tensor, box: float, n_bins: int):
    """Raw P(k) of a real density-contrast mesh (eq. powerspectrum)."""
    n = delta.shape[0]
    return power_spectrum_from_k(fourier.rfft3(delta), n, box, n_bins)


def shell_mask(n: int, centre: float, width: float) -> torch.Tensor:
    """1_{S}: (2c - w)^2 <= 4|n|^2 < (2c + w)^2 on the r2c grid (float64 decision)."""
    s4 = 4.0 * mode_norm_sq(n).double()
    lo = (2.0 * centre - width) ** 2
    hi = (2.0 * centre + width) ** 2
    return ((s4 >= lo) & (s4 < hi)).double()


def bispectrum(delta: torch.Tensor, box: float, centres, width: float, triangles):
    """FFT shell estimator.  ``triangles`` lists (a, b, c) shell ids.
    Returns (B [(Mpc/h)^6], N_tri float64 (sum_x I_a I_b I_c times N^6))."""
    n = delta.shape[0]
    dhat = fourier.rfft3(delta)
    used = sorted({s for tri in triangles for s in tri})
    fields, inds = {}, {}
    for s in used:
        m = shell_mask(n, centres[s], width)
        fields[s] = fourier.irfft3(dhat * m, n)
        inds[s] = fourier.irfft3(m.to(torch.complex128), n)
    vol = box ** 3
    bk, ntri = [], []
    for a, b, c in triangles:
        num = float((fields[a] * fields[b] * fields[c]).sum())
        den = float((inds[a] * inds[b] * inds[c]).sum())
        bk.append(vol ** 2 / n ** 9 * num / den if den != 0.0 else 0.0)
        ntri.append(den * n ** 6)
    return torch.tensor(bk, dtype=torch.float64), torch.tensor(ntri, dtype=torch.float64)


def brute_bispectrum(delta: torch.Tensor, box: float, centres, width: float, triangles):
    """Direct sum over closed triangles of full-cube modes (pin for tiny meshes)."""
    n = delta.shape[0]
    full = torch.fft.fftn(delta.to(torch.complex128))
    f = torch.fft.fftfreq(n, d=1.0 / n).round().long().tolist()
    modes = [(a, b, c) for a in f for b in f for c in f]
    def inshell(m, s):
        r2 = 4.0 * (m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
        return (2 * centres[s] - width) ** 2 <= r2 < (2 * centres[s] + width) ** 2
    def fold(v):
        v = v % n
        return v - n if v >= n // 2 else v
    vol = box ** 3
    out_b, out_n = [], []
    for a, b, c in triangles:
        sa = [m for m in modes if inshell(m, a)]
        sb = [m for m in modes if inshell(m, b)]
        tot, cnt = 0.0 + 0.0j, 0
        for m1 in sa:
            for m2 in sb:
                m3 = tuple(fold(-(m1[d] + m2[d])) for d in range(3))
                if inshell(m3, c):
                    tot += complex(full[m1[0] % n, m1[1] % n, m1[2] % n] * full[m2[0] % n, m2[1] % n, m2[2] % n]
                                   * full[m3[0] % n, m3[1] % n, m3[2] % n])
                    cnt += 1
        out_b.append(vol ** 2 / n ** 9 * tot.real / cnt if cnt else 0.0)
        out_n.append(float(cnt))
    return torch.tensor(out_b, dtype=torch.float64), torch.tensor(out_n, dtype=torch.float64)


def power_spectrum_sparse(modes: torch.Tensor, values: torch.Tensor, n: int, box: float, n_bins: int,
                          values_b: torch.Tensor | None = None):
    """``power_spectrum_from_k`` of an r2c spectrum that vanishes except at the stored
    modes ``modes`` ([M, 3]: n_x, n_y in [-N/2, N/2), n_z in [0, N/2]) with amplitudes
    ``values``; with ``values_b`` (a second spectrum on the same modes) the cross
    spectrum, Re(values conj(values_b)), as ``cross_power_spectrum`` bins it.  Mode
    counts and mean |k| run over every mode, one n_x plane at a time, so no N^3 array
    is formed."""
    full = torch.fft.fftfreq(n, d=1.0 / n).round().long()
    nz = torch.arange(n // 2 + 1, dtype=torch.long)
    wz = torch.full((n // 2 + 1,), 2.0, dtype=torch.float64)
    wz[0] = 1.0
    wz[n // 2] = 1.0
    cnt = torch.zeros(n_bins, dtype=torch.float64)
    sk = torch.zeros(n_bins, dtype=torch.float64)

    def bin_of(s):
        return bin_of_norm2(s, n, n_bins)

    yz = full.view(n, 1) ** 2 + nz.view(1, n // 2 + 1) ** 2
    w_plane = wz.view(1, -1).expand(n, n // 2 + 1).reshape(-1)
    # planes n_x and -n_x hold the same |n|: visit |n_x| once with its multiplicity
    for ax in range(n // 2 + 1):
        mult = 1.0 if ax in (0, n // 2) else 2.0
        s = (ax * ax + yz).reshape(-1)
        b = bin_of(s)
        sel = b >= 0
        cnt.index_add_(0, b[sel], mult * w_plane[sel])
        sk.index_add_(0, b[sel], (mult * w_plane * torch.sqrt(s.double()))[sel])
    m = modes.long()
    s = (m * m).sum(dim=1)
    b = bin_of(s)
    wt = wz[m[:, 2]]
    vb = values if values_b is None else values_b
    p2 = values.real * vb.real + values.imag * vb.imag
    sp = torch.zeros(n_bins, dtype=torch.float64)
    sel = b >= 0
    sp.index_add_(0, b[sel], (wt * p2)[sel])
    kf = 2.0 * math.pi / box
    safe = torch.where(cnt > 0, cnt, torch.ones_like(cnt))
    pk = torch.where(cnt > 0, box ** 3 / n ** 6 * sp / safe, torch.zeros_like(cnt))
    km = torch.where(cnt > 0, kf * sk / safe, torch.zeros_like(cnt))
    return km, pk, cnt.round().long()


def _in_shell(m: torch.Tensor, centre: float, width: float) -> torch.Tensor:
    # the float64 decision of shell_mask on integer modes [..., 3]
    s4 = 4.0 * (m * m).sum(dim=-1).double()
    return (s4 >= (2.0 * centre - width) ** 2) & (s4 < (2.0 * centre + width) ** 2)


def _fold(v: torch.Tensor, n: int) -> torch.Tensor:
    return torch.remainder(v + n // 2, n) - n // 2


def shell_modes(n: int, centre: float, width: float) -> torch.Tensor:
    """Full-cube modes (components in [-N/2, N/2)) of the shell used by ``shell_mask``, [K, 3]."""
    r = min(int(math.ceil(centre + 0.5 * width)) + 1, n // 2)
    ax = torch.arange(-r, min(r, n // 2 - 1) + 1, dtype=torch.long)
    g = torch.stack(torch.meshgrid(ax, ax, ax, indexing="ij"), dim=-1).reshape(-1, 3)
    return g[_in_shell(g, centre, width)]


def triangle_count(n: int, centres, width: float, tri) -> int:
    """N_tri of ``bispectrum``: ordered (p, q, r) in S_a x S_b x S_c with p + q + r = 0
    modulo N, counted by brute force (enumerating the two smallest shells)."""
    shells = [shell_modes(n, centres[s], width) for s in tri]
    order = sorted(range(3), key=lambda i: shells[i].shape[0])
    sp, sq = shells[order[0]], shells[order[1]]
    ck = centres[tri[order[2]]]
    total = 0
    for i0 in range(0, sp.shape[0], 256):
        p = sp[i0:i0 + 256]
        r = _fold(-(p.unsqueeze(1) + sq.unsqueeze(0)), n)
        total += int(_in_shell(r, ck, width).sum())
    return total


def bispectrum_numerator_sparse(modes: torch.Tensor, values: torch.Tensor, n: int, centres, width: float, tri):
    """sum over ordered closed triples (p + q + r = 0 modulo N) with p in S_a, q in S_b,
    r in S_c of dhat(p) dhat(q) dhat(r), for a full-cube spectrum that vanishes except
    at ``modes`` (components in [-N/2, N/2)) with amplitudes ``values``."""
    m = modes.long()
    ia, ib, ic = (_in_shell(m, centres[s], width) for s in tri)
    closed = (_fold(m.view(-1, 1, 1, 3) + m.view(1, -1, 1, 3) + m.view(1, 1, -1, 3), n) == 0).all(dim=-1)
    mask = closed & ia.view(-1, 1, 1) & ib.view(1, -1, 1) & ic.view(1, 1, -1)
    prod = values.view(-1, 1, 1) * values.view(1, -1, 1) * values.view(1, 1, -1)
    return complex(prod[mask].sum()) if bool(mask.any()) else 0j


def bin_of_norm2(s: torch.Tensor, n: int, n_bins: int) -> torch.Tensor:
    """Bin of integer |n|^2 values under the rule of ``pk_bin_index`` (-1 outside every
    bin), without forming the N^3 grid: the b with N^2 (2b+1)^2 <= 16 n_bins^2 |n|^2 <
    N^2 (2b+3)^2 from a float guess floor((4 n_bins |n| / N - 1) / 2) settled by the
    integer inequalities."""
    q = 16 * n_bins * n_bins * s
    b = torch.floor((4.0 * n_bins * torch.sqrt(s.double()) / n - 1.0) / 2.0).long()
    for _ in range(2):
        b = torch.where(n * n * (2 * b + 1) ** 2 > q, b - 1, b)
        b = torch.where(n * n * (2 * b + 3) ** 2 <= q, b + 1, b)
    return torch.where((b >= 0) & (b < n_bins), b, torch.full_like(b, -1))


def cross_power_spectrum(delta_a: torch.Tensor, delta_b: torch.Tensor, box: float, n_bins: int):
    """(k_mean, P_ab, n_modes): the cross spectrum of two meshes of one box,
    <delta_a(k) delta_b(k)*> = (2 pi)^3 delta_D(0) P_ab, i.e. (V/N^6) <Re(a_hat conj(b_hat))>
    over the P(k) bins (cross power of the combined and Newtonian fields; the halo-
    matter cross power of the bias fits, Sec. 5, with matter fields as proxies)."""
    n = delta_a.shape[0]
    ah, bh = fourier.rfft3(delta_a.to(torch.float64)), fourier.rfft3(delta_b.to(torch.float64))
    b = pk_bin_index(n, n_bins).reshape(-1)
    wt = fourier.r2c_weights(n).expand(n, n, n // 2 + 1).reshape(-1)
    cross = (ah.real * bh.real + ah.imag * bh.imag).reshape(-1)
    kmag = torch.sqrt(mode_norm_sq(n).double()).reshape(-1)
    sel = b >= 0
    cnt = torch.zeros(n_bins, dtype=torch.float64).index_add(0, b[sel], wt[sel])
    sp = torch.zeros(n_bins, dtype=torch.float64).index_add(0, b[sel], (wt * cross)[sel])
    sk = torch.zeros(n_bins, dtype=torch.float64).index_add(0, b[sel], (wt * kmag)[sel])
    safe = torch.where(cnt > 0, cnt, torch.ones_like(cnt))
    pk = torch.where(cnt > 0, box ** 3 / n ** 6 * sp / safe, torch.zeros_like(cnt))
    km = torch.where(cnt > 0, 2.0 * math.pi / box * sk / safe, torch.zeros_like(cnt))
    return km, pk, cnt.round().long()


def bias_fit(k: torch.Tensor, ratio: torch.Tensor, n_modes: torch.Tensor, k_cut: float, calh: float,
             skip: int = 2, with_k2: bool = True):
    """Scale-dependent linear bias (eq. b1 with the scale dependence of Sec. 5):
    ratio(k) = b1 + b1_GR calH^2 / k^2 [+ c2 k^2], fitted by weighted least squares
    (weights: mode counts, reading) over the bins with 0 < k < k_cut after dropping
    the first ``skip`` of them (the paper drops the first two points).  calH in h/Mpc.
    Returns (b1, b1_GR, c2) (c2 = 0 without the k^2 term)."""
    sel = [i for i in range(k.shape[0]) if n_modes[i] > 0 and 0.0 < float(k[i]) < k_cut]
    sel = sel[skip:]
    kk = k[sel].to(torch.float64)
    cols = [torch.ones_like(kk), calh * calh / (kk * kk)] + ([kk * kk] if with_k2 else [])
    a = torch.stack(cols, dim=1)
    w = torch.sqrt(n_modes[sel].to(torch.float64)).view(-1, 1)
    sol = torch.linalg.lstsq(a * w, ratio[sel].to(torch.float64).view(-1, 1) * w).solution.view(-1)
    return float(sol[0]), float(sol[1]), float(sol[2]) if with_k2 else 0.0
