"""Planted mistakes in the oracle must fail its pins (CPU only, no GPU).

Each case rewrites one or two lines of an oracle function into a plausible slip: a
sign, a wrong neighbour or slice, a dropped term or factor, a missing conjugate, a
transposed operand, a wrong recurrence coefficient.  The rewritten function is
compiled from the oracle's own source, installed wherever the original is bound
(the oracle's modules and the pin modules) for the duration of the case, and the
pins of the modules that cover it run in definition order until one fails.  The
case passes when some pin fails.

A rewrite of M is applied to both of the oracle's builders of M, so the pin that
has to catch it is an independent one (closed form, invariance, finite
differences, brute force, a number the paper prints), not the comparison of the
two builders.
"""
import __future__
import importlib
import inspect
import itertools
import sys
import textwrap

import numpy as np
import pytest

import oracle
import oracle.correlators
import oracle.ed
import oracle.force
import oracle.hasenbusch
import oracle.hmc
import oracle.multishift
import oracle.operator
import oracle.solve

PINS = ["test_oracle_pins", "test_oracle_hasenbusch", "test_oracle_multishift", "test_oracle_hmc",
        "test_oracle_ed", "test_oracle_correlators"]

# (case id, "module:qualified name", [(old text, new text, occurrence)], pin modules)
OP = ["test_oracle_pins"]
CASES = [
    # eq. (ferm_op): the temporal hops
    ("M periodic A hop", "oracle.operator:build_M",
     [("np.where(t == 0, -1.0, 1.0)", "np.where(t == 0, 1.0, 1.0)", 0)], OP),
    ("M periodic B hop", "oracle.operator:build_M",
     [("np.where(t == lat.Nt - 1, -1.0, 1.0)", "np.where(t == lat.Nt - 1, 1.0, 1.0)", 0)], OP),
    ("M A phase sign", "oracle.operator:build_M",
     [("np.exp(1j * phi[t, 0, i, j])", "np.exp(-1j * phi[t, 0, i, j])", 0)], OP),
    ("M B phase sign", "oracle.operator:build_M",
     [("np.exp(-1j * phi[t, 1, i, j])", "np.exp(1j * phi[t, 1, i, j])", 0)], OP),
    ("M A phase from slice t-1", "oracle.operator:build_M",
     [("phi[t, 0, i, j]", "phi[tm, 0, i, j]", 0)], OP),
    ("M B phase from slice t+1", "oracle.operator:build_M",
     [("phi[t, 1, i, j]", "phi[tp, 1, i, j]", 0)], OP),
    ("M A hop forward in time", "oracle.operator:build_M",
     [("tm = (t - 1) % lat.Nt", "tm = (t + 1) % lat.Nt", 0)], OP),
    ("M B hop backward in time", "oracle.operator:build_M",
     [("tp = (t + 1) % lat.Nt", "tp = (t - 1) % lat.Nt", 0)], OP),
    ("M B hop sign", "oracle.operator:build_M",
     [("vals.append(-sgn_p *", "vals.append(sgn_p *", 0)], OP),
    ("M A diagonal sign", "oracle.operator:build_M",
     [("np.full(a.shape, -1.0 + 0j)", "np.full(a.shape, 1.0 + 0j)", 0)], OP),
    ("M staggered mass sign on A", "oracle.operator:build_M",
     [("- lat.ms_t)", "+ lat.ms_t)", 0)], OP),
    ("M staggered mass dropped on B", "oracle.operator:build_M",
     [("- lat.ms_t)", ")", 1)], OP),
    # eq. (ferm_op): the bonds
    ("M bond to cell i+1", "oracle.operator:build_M",
     [("((i - 1) % lat.L1, j)", "((i + 1) % lat.L1, j)", 0)], OP),
    ("M bond to cell j+1", "oracle.operator:build_M",
     [("(i, (j - 1) % lat.L2)", "(i, (j + 1) % lat.L2)", 0)], OP),
    ("M bond to cell (i-1, j-1)", "oracle.operator:build_M",
     [("(i, (j - 1) % lat.L2)", "((i - 1) % lat.L1, (j - 1) % lat.L2)", 0)], OP),
    ("M hopping sign", "oracle.operator:build_M",
     [("np.full(a.shape, -lat.kappa_t + 0j)", "np.full(a.shape, lat.kappa_t + 0j)", 0)], OP),
    ("M hopping one way only", "oracle.operator:build_M",
     [("rows.append(nb); cols.append(a); vals.append(hop)", "pass", 0)], OP),
    ("M transposed", "oracle.operator:build_M", [("return M.tocsr()", "return M.T.tocsr()", 0)], OP),
    ("M conjugated", "oracle.operator:build_M", [("return M.tocsr()", "return M.conj().tocsr()", 0)], OP),
    # the adjoint and the normal operator of Sec. 3
    ("Mdag without conjugate", "oracle.operator:apply_Mdag",
     [("Mh = M.conj().T.tocsr()", "Mh = M.T.tocsr()", 0)], OP),
    ("Mdag without transpose", "oracle.operator:apply_Mdag",
     [("Mh = M.conj().T.tocsr()", "Mh = M.conj().tocsr()", 0)], OP),
    ("normal operator is Mdag M", "oracle.operator:NormalOperator",
     [("self.M @ (self.Mh @ x)", "self.Mh @ (self.M @ x)", 0),
      ("Md @ Md.conj().T", "Md.conj().T @ Md", 0)], OP),
    ("normal operator shift sign", "oracle.operator:NormalOperator",
     [("+ self.mu2 * x", "- self.mu2 * x", 0), ("+ self.mu2 * np.eye", "- self.mu2 * np.eye", 0)], OP),
    # eqs. (p_dot), (eta_xi): the force and the action
    ("dM/dphi A link forward", "oracle.force:dM_dphi_entries",
     [("np.where(isA, (t - 1) % lat.Nt", "np.where(isA, (t + 1) % lat.Nt", 0)], OP),
    ("dM/dphi B link backward", "oracle.force:dM_dphi_entries",
     [("(t + 1) % lat.Nt)", "(t - 1) % lat.Nt)", 0)], OP),
    ("dM/dphi periodic A", "oracle.force:dM_dphi_entries",
     [("np.where(t == 0, -1.0, 1.0)", "np.where(t == 0, 1.0, 1.0)", 0)], OP),
    ("dM/dphi periodic B", "oracle.force:dM_dphi_entries",
     [("np.where(t == lat.Nt - 1, -1.0, 1.0)", "np.where(t == lat.Nt - 1, 1.0, 1.0)", 0)], OP),
    ("dM/dphi B phase sign", "oracle.force:dM_dphi_entries",
     [("1j * sign * np.exp(-1j * ph)", "1j * sign * np.exp(1j * ph)", 0)], OP),
    ("dM/dphi without the factor i", "oracle.force:dM_dphi_entries",
     [("1j * sign * np.exp(1j * ph)", "sign * np.exp(1j * ph)", 0)], OP),
    ("force sign", "oracle.force:force", [("F = -2.0 *", "F = 2.0 *", 0)], OP),
    ("force factor 2 dropped", "oracle.force:force", [("F = -2.0 *", "F = -1.0 *", 0)], OP),
    ("force without conjugate", "oracle.force:force", [("np.conj(e[:, row])", "e[:, row]", 0)], OP),
    ("force imaginary part", "oracle.force:force", [("* x[:, col]).real", "* x[:, col]).imag", 0)], OP),
    ("force eta and xi swapped", "oracle.force:force",
     [("np.conj(e[:, row]) * val[None, :] * x[:, col]", "np.conj(x[:, row]) * val[None, :] * e[:, col]", 0)], OP),
    ("xi = M eta", "oracle.force:xi_from_eta",
     [("apply_Mdag(lat, phi, eta)", "__import__('oracle').operator.apply_M(lat, phi, eta)", 0)], OP),
    ("action imaginary part", "oracle.force:action", [("np.vdot(c.ravel(), e.ravel()).real", "np.vdot(c.ravel(), e.ravel()).imag", 0)], OP),
    # Sec. 3 CG and Algorithm A.1
    ("CG beta inverted", "oracle.solve:cg", [("(rr_new / rr) * p", "(rr / rr_new) * p", 0)], OP),
    ("CG alpha from |q|^2", "oracle.solve:cg", [("np.vdot(p, q).real", "np.vdot(q, q).real", 0)], OP),
    ("CG without restart", "oracle.solve:cg", [("p = r + (rr_new / rr) * p", "p = r.copy()", 0)], OP),
    ("spCG beta inverted", "oracle.solve:_spcg_c64", [("np.float32(rr_new / rr) * p", "np.float32(rr / rr_new) * p", 0)], OP),
    ("A.1 Gram-Schmidt conjugated", "oracle.solve:fgmres_alg_a1",
     [("H[i, j] = np.vdot(V[i], w)", "H[i, j] = np.vdot(w, V[i])", 0)], OP),
    ("A.1 update over v instead of z", "oracle.solve:fgmres_alg_a1",
     [("x = x + y[i] * Z[i]", "x = x + y[i] * V[i]", 0)], OP),
    ("A.1 least squares right-hand side", "oracle.solve:fgmres_alg_a1",
     [("rhs[0] = rnorm", "rhs[0] = 1.0", 0)], OP),
    ("A.1 subdiagonal dropped", "oracle.solve:fgmres_alg_a1",
     [("H[j + 1, j] = _norm(w)", "H[j + 1, j] = 0.0 * _norm(w)", 0)], OP),
    ("A.1 residual estimate as the product of subdiagonals", "oracle.solve:fgmres_alg_a1",
     [("ERR = _norm(e1 - H[: j + 2, : j + 1] @ yj)", "ERR = ERR * H[j + 1, j].real", 0)], OP),
    ("A.1 residual estimate not updated", "oracle.solve:fgmres_alg_a1",
     [("ERR = _norm(e1 - H[: j + 2, : j + 1] @ yj)", "ERR = ERR", 0)], OP),
    ("A.1 one projection per step", "oracle.solve:fgmres_alg_a1",
     [("for i in range(j + 1):\n                w = w - H[i, j] * V[i]",
       "for i in range(j, j + 1):\n                w = w - H[i, j] * V[i]", 0)], OP),
    # Sec. 5.1 Hasenbusch split
    ("Hasenbusch heat-bath mass", "oracle.hasenbusch:heatbath",
     [("mass_of(lat, mts, i - 1)), phi, rho[i])", "mass_of(lat, mts, i)), phi, rho[i])", 0)],
     ["test_oracle_hasenbusch"]),
    ("Hasenbusch last heat-bath mass", "oracle.hasenbusch:heatbath",
     [("mass_of(lat, mts, n - 1)", "mass_of(lat, mts, n - 2)", 0)], ["test_oracle_hasenbusch"]),
    ("Hasenbusch denominator mass", "oracle.hasenbusch:term",
     [("(n - 1) if i == n else (i - 1)", "(n - 1) if i == n else i", 0)], ["test_oracle_hasenbusch"]),
    ("Hasenbusch ratio force without chi", "oracle.hasenbusch:term",
     [("xi if i == n else xi - chi_i", "xi", 0)], ["test_oracle_hasenbusch"]),
    ("Hasenbusch numerator operator dagger", "oracle.hasenbusch:term",
     [("w = apply_M(lattice_with_mass(lat, mass_of(lat, mts, i)), phi, chi_i)",
       "w = apply_Mdag(lattice_with_mass(lat, mass_of(lat, mts, i)), phi, chi_i)", 0)], ["test_oracle_hasenbusch"]),
    # Sec. 5.2 integrator, Sec. 2 Hamiltonian
    ("Omelyan middle kick", "oracle.hmc:Integrator",
     [("self.kick(k, (1 - 2 * z) * h)\n", "self.kick(k, (1 - z) * h)\n", 0)], ["test_oracle_hmc"]),
    ("Omelyan split half step", "oracle.hmc:Integrator",
     [("self.kick(k, (1 - 2 * z) * h / 2)", "self.kick(k, (1 - 2 * z) * h)", 0)], ["test_oracle_hmc"]),
    ("nested level drift", "oracle.hmc:Integrator",
     [("self.drift(h / 2)", "self.drift(h)", 0)], ["test_oracle_hmc"]),
    ("gauge force sign", "oracle.hmc:level_force",
     [("F = F + np.asarray(phi) / U_t", "F = F - np.asarray(phi) / U_t", 0)], ["test_oracle_hmc"]),
    ("gauge action factor", "oracle.hmc:gauge_action",
     [("0.5 * float(np.sum(p * p)) / U_t", "float(np.sum(p * p)) / U_t", 0)], ["test_oracle_hmc"]),
    ("Metropolis direction", "oracle.hmc:hmc_update", [("u < np.exp(-dH)", "u < np.exp(dH)", 0)], ["test_oracle_hmc"]),
    ("nested odd half step misplaced", "oracle.hmc:Integrator",
     [("            for _ in range(j):\n                self._step(k + 1, self.H[k + 1])\n            if odd:\n"
       "                self._half_step(k + 1, self.H[k + 1], first=True)",
       "            if odd:\n                self._half_step(k + 1, self.H[k + 1], first=True)\n"
       "            for _ in range(j):\n                self._step(k + 1, self.H[k + 1])", 0)], ["test_oracle_hmc"]),
    ("nested odd ratio dropped", "oracle.hmc:Integrator", [("j, odd = divmod(r, 2)", "j, odd = r // 2, 0", 0)],
     ["test_oracle_hmc"]),
    ("kinetic energy factor", "oracle.hmc:kinetic", [("0.5 * float(np.sum(p * p))", "float(np.sum(p * p))", 0)],
     ["test_oracle_hmc"]),
    ("true residual not relative", "oracle.solve:true_rel_residual",
     [("return _norm(bf - A(xf)) / _norm(bf)", "return _norm(bf - A(xf))", 0)], OP),
    ("M^-1 solve with the adjoint", "oracle.hasenbusch:solve_M",
     [("x = spla.spsolve(build_M(lat, phi).tocsc(), bf.ravel())",
       "x = spla.spsolve(build_M(lat, phi).conj().T.tocsc(), bf.ravel())", 0)], ["test_oracle_hasenbusch"]),
    # Sec. 5.1, 6.1 shifts and spectra
    ("CG-M alpha ratio inverted", "oracle.multishift:cg_multishift",
     [("a_s = a * z_next / z_cur[s]", "a_s = a * z_cur[s] / z_next", 0)], ["test_oracle_multishift"]),
    ("CG-M beta ratio not squared", "oracle.multishift:cg_multishift",
     [("(z_next / z_cur[s]) ** 2", "(z_next / z_cur[s])", 0)], ["test_oracle_multishift"]),
    ("CG-M shift sign", "oracle.multishift:cg_multishift", [("(1.0 + sg * a)", "(1.0 - sg * a)", 0)],
     ["test_oracle_multishift"]),
    ("Lanczos diagonal", "oracle.multishift:lanczos_tridiagonal",
     [("bt[j - 1] / a[j - 1]", "bt[j - 1] / a[j]", 0)], ["test_oracle_multishift"]),
    ("Lanczos off-diagonal", "oracle.multishift:lanczos_tridiagonal",
     [("np.sqrt(bt[j]) / a[j]", "bt[j] / a[j]", 0)], ["test_oracle_multishift"]),
    ("Hasenbusch masses exponent", "oracle.multishift:hasenbusch_masses",
     [("((i + 1) / (n + 1))", "((i + 1) / n)", 0)], ["test_oracle_multishift"]),
    ("spectrum extremes swapped", "oracle.multishift:spectrum_extremes",
     [("return float(ev[0]), float(ev[-1])", "return float(ev[-1]), float(ev[0])", 0)], ["test_oracle_multishift"]),
    # Sec. 7.2 exact diagonalisation and correlators
    ("ED hopping not symmetric", "oracle.ed:hopping", [("h[b, a] -= kappa", "h[b, a] += kappa", 0)],
     ["test_oracle_ed"]),
    ("ED without Jordan-Wigner signs", "oracle.ed:_annihilators",
     [("sign = np.array([(-1) ** bin(int(x)).count(\"1\") for x in lower])", "sign = np.ones(dim)", 0)],
     ["test_oracle_ed", "test_oracle_correlators"]),
    ("ED interaction on one spin", "oracle.ed:hamiltonian",
     [("(n[x] - 0.5 * I) @ (n[ns + x] - 0.5 * I)", "(n[x] - 0.5 * I) @ (n[x] - 0.5 * I)", 0)],
     ["test_oracle_ed"]),
    ("ED interaction without half filling shift", "oracle.ed:hamiltonian",
     [("(n[x] - 0.5 * I) @ (n[ns + x] - 0.5 * I)", "n[x] @ n[ns + x]", 0)], ["test_oracle_ed"]),
    ("ED thermal weight", "oracle.ed:thermal_correlator",
     [("wm = np.exp(-(beta - tau) * ev)", "wm = np.exp(-beta * ev)", 0)],
     ["test_oracle_ed", "test_oracle_correlators"]),
    ("quasi-particle level without degeneracy sum", "oracle.ed:quasiparticle_energies",
     [("levels[-1][1] += w[j]", "pass", 0)], ["test_oracle_ed"]),
    ("quasi-particle energy not relative to the ground state", "oracle.ed:quasiparticle_energies",
     [("float(E - ev[0])", "float(E)", 0)], ["test_oracle_ed"]),
    ("fit window ignored", "oracle.correlators:fit_energy", [("& (C > 0)", "& (C > 0) | (tau >= 0)", 0)],
     ["test_oracle_correlators"]),
    ("correlator wrap sign", "oracle.correlators:propagator_correlator",
     [("sgn = -1.0 if t0 + k >= lat.Nt else 1.0", "sgn = 1.0", 0)], ["test_oracle_correlators"]),
    ("correlator overall sign", "oracle.correlators:propagator_correlator",
     [("C[k] += -sgn *", "C[k] += sgn *", 0)], ["test_oracle_correlators"]),
    ("fit slope sign", "oracle.correlators:fit_energy", [("return float(-slope)", "return float(slope)", 0)],
     ["test_oracle_correlators"]),
]


def _replace_nth(src, old, new, n):
    pos = -1
    for _ in range(n + 1):
        pos = src.find(old, pos + 1)
        assert pos >= 0, f"pattern not found: {old!r}"
    return src[:pos] + new + src[pos + len(old):]


def _mutant(target, edits):
    modname, qual = target.split(":")
    mod = importlib.import_module(modname)
    orig = getattr(mod, qual)
    src = textwrap.dedent(inspect.getsource(orig))
    for old, new, n in edits:
        src = _replace_nth(src, old, new, n)
    ns = dict(vars(mod))
    exec(compile(src, f"<mutant {target}>", "exec", flags=__future__.annotations.compiler_flag,
                 dont_inherit=True), ns)
    return orig, ns[qual]


def _install(monkeypatch, orig, new):
    """Bind `new` wherever `orig` is bound in the oracle's and the pins' modules."""
    for name, mod in list(sys.modules.items()):
        if not (name == "oracle" or name.startswith("oracle.") or "test_oracle_" in name):
            continue
        for k, v in list(vars(mod).items()):
            if v is orig:
                monkeypatch.setattr(mod, k, new)


def _params(fn):
    grids = []
    for mark in getattr(fn, "pytestmark", []):
        if mark.name != "parametrize":
            continue
        names, values = mark.args[0], mark.args[1]
        names = [x.strip() for x in names.split(",")] if isinstance(names, str) else list(names)
        rows = []
        for v in values:
            if type(v).__name__ == "ParameterSet":      # pytest.param(...)
                v = tuple(v.values)
            elif len(names) == 1:
                v = (v,)
            rows.append(dict(zip(names, v)))
        grids.append(rows)
    for combo in itertools.product(*grids):
        kw = {}
        for d in combo:
            kw.update(d)
        yield kw


def _first_failing_pin(modnames):
    for modname in modnames:
        mod = sys.modules.get(modname) or importlib.import_module(modname)
        for name, fn in list(vars(mod).items()):
            if not (name.startswith("test_") and callable(fn)):
                continue
            for kw in _params(fn):
                try:
                    with np.errstate(all="ignore"):
                        fn(**kw)
                except Exception as e:  # an assertion, a LinAlgError, a shape error: the pin fails
                    return f"{modname}.{name}{kw or ''}: {type(e).__name__}"
    return None


@pytest.fixture(scope="module", autouse=True)
def _pin_modules():
    for m in PINS:
        importlib.import_module(m)


def test_unmutated_oracle_passes_the_pins():
    assert _first_failing_pin(PINS) is None


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_fails_a_pin(monkeypatch, case):
    _, target, edits, pins = case
    orig, new = _mutant(target, edits)
    _install(monkeypatch, orig, new)
    if target == "oracle.operator:build_M":
        _install(monkeypatch, oracle.operator.build_M_dense_loops, lambda lat, phi: new(lat, phi).toarray())
    caught = _first_failing_pin(pins)
    assert caught is not None, f"no pin fails with the planted mistake {case[0]!r}"
