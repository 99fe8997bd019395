"""Element-wise comparison of GPU fields with the FP64 oracle's (shared by the GPU tests).

Bars, by population storage.  The velocity bars are the stated accuracy
targets: 1e-5 in FP32 and 1e-3 in FP16 storage; BF16 keeps 8 mantissa bits,
8x fewer than FP16's 11, and is held to 1e-2.

* u, relative L2 over all sites and components: ||u - u_o|| / ||u_o|| < bar.
* u, per element: max |u - u_o| / max |u_o| < 10 bar.  This check is there for
  localised defects (a wrong value at a tile edge or a wrapped halo is an
  error of the order of the velocity itself, far above 10 bar), while the
  rounding of a correct kernel concentrates at the interface cells, where the
  surface-tension and pressure forces are differences of large terms: the
  observed max / L2 ratio is 1-5 in every case.
* p, per element: max |p - p_o| < bar * max |p_o - mean p_o| + floor, with
  floor = 2^-22 max |p_o| + eps_s (rho_max c_s^2) (max |p*_o - mean p*_o| + 6 max |u_o|):
  two FP32 ulps of the returned p = p* rho c_s^2, plus the storage rounding
  of the populations that carry p*: a stored h_i = f_i / w_i - P0 is about
  p* - P0 + 3 c_i.u (|c_i| <= sqrt 3), rounded with unit roundoff eps_s
  (2^-24 FP32, 2^-11 FP16, 2^-8 BF16), and p* - P0 = sum_i w_i h_i.  The
  mean of p*_o stands in for the gauge P0 (the mean pressure of every case).
* rho, per element: max |rho - rho_o| < 4 * 2^-24 max rho_o + drho * phi_bar
  (the FP32 output's rounding plus the density jump times the phi error bound).
"""
import numpy as np

U_BAR = {"f32": 1e-5, "f16": 1e-3, "bf16": 1e-2}
EPS_STORE = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}
ELEMENT_FACTOR = 10.0


def errors(m, mo, storage="f32"):
    """Error measures of GPU fields m against oracle fields mo (numpy, FP64)."""
    du = m["u"] - mo["u"]
    out = {
        "u_rel_l2": float(np.linalg.norm(du) / np.linalg.norm(mo["u"])),
        "u_max_rel": float(np.abs(du).max() / np.abs(mo["u"]).max()),
    }
    if "p" in m and "p" in mo and "rho" in mo:
        po, rho = mo["p"], mo["rho"]
        pstar = po / (rho / 3.0)
        out["p_max_abs"] = float(np.abs(m["p"] - po).max())
        out["p_var"] = float(np.abs(po - po.mean()).max())
        out["p_floor"] = float(2.0 ** -22 * np.abs(po).max() + EPS_STORE[storage] * (rho.max() / 3.0) *
                               (np.abs(pstar - pstar.mean()).max() + 6.0 * np.abs(mo["u"]).max()))
    if "rho" in m and "rho" in mo:
        out["rho_max_abs"] = float(np.abs(m["rho"] - mo["rho"]).max())
        out["rho_max"] = float(np.abs(mo["rho"]).max())
    if "phi" in m and "phi" in mo:
        out["phi_max_abs"] = float(np.abs(m["phi"] - mo["phi"]).max())
    return out


def check(m, mo, storage="f32", label="", u_bar=None, p_bar=None, phi_bar=None, drho=0.0, p=True):
    """Assert the element-wise bars above (u_bar / p_bar / phi_bar override the
    storage defaults; p_bar defaults to u_bar); returns the error measures."""
    ub = U_BAR[storage] if u_bar is None else u_bar
    pb = ub if p_bar is None else p_bar
    e = errors(m, mo, storage)
    msg = (f"{label} [{storage}] u rel L2 {e['u_rel_l2']:.3e} (bar {ub:.3g}), u max/max|u| "
           f"{e['u_max_rel']:.3e} (bar {ELEMENT_FACTOR * ub:.3g})")
    ok = e["u_rel_l2"] < ub and e["u_max_rel"] < ELEMENT_FACTOR * ub
    if p and "p_max_abs" in e:
        lim = pb * e["p_var"] + e["p_floor"]
        msg += (f", p max abs {e['p_max_abs']:.3e} (bar {lim:.3e}: {pb:.3g} x var {e['p_var']:.2e} + "
                f"floor {e['p_floor']:.2e})")
        ok = ok and e["p_max_abs"] <= lim
    if "rho_max_abs" in e:
        lim = 4 * 2.0 ** -24 * e["rho_max"] + drho * (phi_bar or 0.0)
        msg += f", rho max abs {e['rho_max_abs']:.3e} (bar {lim:.2e})"
        ok = ok and e["rho_max_abs"] <= lim
    if phi_bar is not None and "phi_max_abs" in e:
        msg += f", phi max abs {e['phi_max_abs']:.3e} (bar {phi_bar:g})"
        ok = ok and e["phi_max_abs"] < phi_bar
    print(msg, flush=True)
    assert ok, msg
    return e
