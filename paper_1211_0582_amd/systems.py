"""Front end of run-time compiled systems: a hyperbolic system written as
flux expressions, turned into the C++ `struct System` that the library
compiles at run time (dg_setup_system) -- the paper's user-level flux
description and run-time code generation (Section 4; the flux figure of
Section 5 writes the Maxwell flux the same way, in terms of the interior and
exterior traces and the normal).

A system is described by
  * ``fields``: field names, in state-array order;
  * ``volume_flux``: for each direction "x", "y", "z" the components of
    F_d(u) as expressions in the field names (absent components are zero);
  * ``numerical_flux``: for each field the expression of n.F - (n.F)* (the
    term the scheme lifts), in the interior values ``<name>_m``, exterior
    values ``<name>_p``, the outward normal ``nx``, ``ny``, ``nz`` and the
    flux parameter ``alpha``;
  * ``boundary``: for each boundary condition code the exterior state as
    expressions in ``<name>_m``, ``nx``, ``ny``, ``nz`` (codes not listed
    get a zero exterior);
  * optionally ``volume_defs`` and ``face_defs``: named intermediate
    expressions, in order, usable in the volume flux (over the field names)
    and in the numerical flux (over the face names) -- e.g. velocity and
    pressure of a nonlinear system.
A nonlinear volume flux is collocated: the kernel differentiates the nodal
values of F_d(u) (the nodal DG form).
Expressions may use numbers, + - * /, unary minus, parentheses and the
functions abs, sqrt, min, max.  They are parsed with Python's own parser,
checked against this grammar and emitted as C++; constants the compiler can
see (a zero flux-matrix entry, a field a boundary state does not touch) then
cost nothing in the kernel.

This module only writes source text; everything it describes runs in the
library's compiled kernel.
"""
from __future__ import annotations

import ast

import numpy as np

from . import dg

_FUNCS = {"abs": "dg_abs", "sqrt": "dg_sqrt", "min": "dg_min", "max": "dg_max"}

_PRELUDE = """template <typename T> __device__ inline T dg_abs(T x) { return x < T(0) ? -x : x; }
template <typename T> __device__ inline T dg_min(T a, T b) { return a < b ? a : b; }
template <typename T> __device__ inline T dg_max(T a, T b) { return a < b ? b : a; }
template <typename T> __device__ inline T dg_sqrt(T x) {
  if constexpr (sizeof(T) == 8) return __builtin_sqrt(x); else return __builtin_sqrtf(x);
}
"""


class ExpressionError(ValueError):
    pass


def _emit(expr: str, names: dict) -> str:
    """C++ text of a flux expression; ``names`` maps allowed identifiers to C++."""
    try:
        tree = ast.parse(expr, mode="eval")
    except SyntaxError as e:
        raise ExpressionError(f"cannot parse {expr!r}: {e}") from None

    def go(n):
        if isinstance(n, ast.Expression):
            return go(n.body)
        if isinstance(n, ast.Constant) and isinstance(n.value, (int, float)) and not isinstance(n.value, bool):
            return f"T({float(n.value)!r})"
        if isinstance(n, ast.Name):
            if n.id not in names:
                raise ExpressionError(f"unknown name {n.id!r} in {expr!r}")
            return names[n.id]
        if isinstance(n, ast.UnaryOp) and isinstance(n.op, (ast.USub, ast.UAdd)):
            return ("-" if isinstance(n.op, ast.USub) else "+") + "(" + go(n.operand) + ")"
        if isinstance(n, ast.BinOp) and isinstance(n.op, (ast.Add, ast.Sub, ast.Mult, ast.Div)):
            op = {ast.Add: "+", ast.Sub: "-", ast.Mult: "*", ast.Div: "/"}[type(n.op)]
            return "(" + go(n.left) + " " + op + " " + go(n.right) + ")"
        if isinstance(n, ast.Call) and isinstance(n.func, ast.Name) and n.func.id in _FUNCS and not n.keywords:
            nargs = 1 if n.func.id in ("abs", "sqrt") else 2
            if len(n.args) != nargs:
                raise ExpressionError(f"{n.func.id} takes {nargs} argument(s) in {expr!r}")
            return _FUNCS[n.func.id] + "<T>(" + ", ".join(go(a) for a in n.args) + ")"
        raise ExpressionError(f"unsupported construct {ast.dump(n)[:60]} in {expr!r}")

    return go(tree)


class SystemSpec:
    def __init__(self, name, fields, volume_flux, numerical_flux, boundary, volume_defs=(), face_defs=()):
        self.name = name
        self.volume_defs = tuple(volume_defs)
        self.face_defs = tuple(face_defs)
        self.fields = tuple(fields)
        if len(set(self.fields)) != len(self.fields) or not 1 <= len(self.fields) <= 12:
            raise ValueError("need 1..12 distinct field names")
        self.volume_flux = {d: dict(volume_flux.get(d, {})) for d in ("x", "y", "z")}
        self.numerical_flux = dict(numerical_flux)
        self.boundary = {int(k): dict(v) for k, v in boundary.items()}
        for d, comps in self.volume_flux.items():
            for f in comps:
                if f not in self.fields:
                    raise ValueError(f"volume flux {d}: unknown field {f!r}")
        for f in self.numerical_flux:
            if f not in self.fields:
                raise ValueError(f"numerical flux: unknown field {f!r}")

    @property
    def M(self):
        return len(self.fields)

    def source(self) -> str:
        """The generated C++ (struct System) for the library's kernel template."""
        M = self.M
        idx = {f: i for i, f in enumerate(self.fields)}
        vol_names = {f: f"u[{i}]" for f, i in idx.items()}
        vol_defs = []
        for dn, de in self.volume_defs:
            vol_defs.append(f"    const T v_{dn} = {_emit(de, vol_names)};")
            vol_names[dn] = f"v_{dn}"
        face = {"nx": "nx", "ny": "ny", "nz": "nz"}
        flux_names = dict(face, alpha="alpha", **{f + "_m": f"um[{i}]" for f, i in idx.items()},
                          **{f + "_p": f"up[{i}]" for f, i in idx.items()})
        bnd_names = dict(face, **{f + "_m": f"um[{i}]" for f, i in idx.items()})
        face_defs = []
        for dn, de in self.face_defs:
            face_defs.append(f"    const T f_{dn} = {_emit(de, flux_names)};")
            flux_names[dn] = f"f_{dn}"
        lines = [f"// generated from the flux description of the system {self.name!r}", _PRELUDE, "struct System {",
                 f"  static constexpr int M = {M};",
                 "  template <typename T>",
                 f"  __device__ static inline void volume(const T (&m)[3], const T (&u)[{M}], T (&x)[{M}]) {{"]
        lines += vol_defs
        for f in self.fields:
            terms = []
            for k, d in enumerate(("x", "y", "z")):
                e = self.volume_flux[d].get(f)
                if e is not None:
                    terms.append(f"m[{k}] * {_emit(e, vol_names)}")
            rhs = "-(" + " + ".join(terms) + ")" if terms else "T(0)"
            lines.append(f"    x[{idx[f]}] = {rhs};  // {f}")
        lines += ["  }", "  template <typename T>",
                  f"  __device__ static inline void exterior(int code, T nx, T ny, T nz, const T (&um)[{M}], "
                  f"T (&up)[{M}]) {{",
                  "    (void)nx; (void)ny; (void)nz; (void)um;", "    switch (code) {"]
        for code in sorted(self.boundary):
            lines.append(f"      case {code}:")
            for f in self.fields:
                e = self.boundary[code].get(f)
                lines.append(f"        up[{idx[f]}] = {_emit(e, bnd_names) if e is not None else 'T(0)'};")
            lines.append("        return;")
        lines += ["      default:", f"        for (int c = 0; c < {M}; ++c) up[c] = T(0);", "    }", "  }",
                  "  template <typename T>",
                  f"  __device__ static inline void flux(T nx, T ny, T nz, T alpha, const T (&um)[{M}], "
                  f"const T (&up)[{M}], T (&f)[{M}]) {{",
                  "    (void)nx; (void)ny; (void)nz; (void)alpha; (void)um; (void)up;"]
        lines += face_defs
        for f in self.fields:
            e = self.numerical_flux.get(f)
            lines.append(f"    f[{idx[f]}] = {_emit(e, flux_names) if e is not None else 'T(0)'};  // {f}")
        lines += ["  }", "};", ""]
        return "\n".join(lines)

    def compile_check(self, N: int, precision="fp64", arch="gfx950") -> str:
        """Compiles the generated source for order N without a device; returns the log."""
        return dg.dg_system_compile(self.source(), self.M, N, precision, arch)


class SystemProblem(dg.Problem):
    """A problem of a run-time compiled system (dg_setup_system)."""

    def __init__(self, spec: SystemSpec, N, VX, EToV, precision="fp64", alpha=1.0, face_bc=None, device=-1):
        self.handle = None
        self.spec = spec
        self.handle = dg.dg_setup_system(N, VX, EToV, spec.source(), spec.M, precision, alpha, face_bc, device)
        self.info = dg.dg_info_get(self.handle)

    @property
    def variant(self):
        return "system"


# ---------------------------------------------------------------------------
# Systems written in the front end
# ---------------------------------------------------------------------------
def _dot(a, b):
    return " + ".join(f"{x}*({y})" for x, y in zip(a, b))


def maxwell() -> SystemSpec:
    """(Ex, Ey, Ez, Hx, Hy, Hz) in conservation form: dE/dt - curl H = 0,
    dH/dt + curl E = 0; the upwind flux of the results section, n.F - (n.F)* =
    1/2 (-n x dH) + alpha/2 (n (n.dE) - dE) for E and the dual for H;
    boundary codes 0 conducting, 1 magnetic-conducting, 2 absorbing."""
    vf = {"x": {"Ey": "Hz", "Ez": "-Hy", "Hy": "-Ez", "Hz": "Ey"},
          "y": {"Ex": "-Hz", "Ez": "Hx", "Hx": "Ez", "Hz": "-Ex"},
          "z": {"Ex": "Hy", "Ey": "-Hx", "Hx": "-Ey", "Hy": "Ex"}}
    n = ("nx", "ny", "nz")
    dE = [f"({c}_m - {c}_p)" for c in ("Ex", "Ey", "Ez")]
    dH = [f"({c}_m - {c}_p)" for c in ("Hx", "Hy", "Hz")]
    ndE, ndH = _dot(n, dE), _dot(n, dH)

    def cross(a, b, i):
        j, k = (i + 1) % 3, (i + 2) % 3
        return f"({a[j]}*{b[k]} - {a[k]}*{b[j]})"

    nf = {}
    for i, c in enumerate(("Ex", "Ey", "Ez")):
        nf[c] = f"0.5*(-{cross(n, dH, i)}) + 0.5*alpha*({n[i]}*({ndE}) - {dE[i]})"
    for i, c in enumerate(("Hx", "Hy", "Hz")):
        nf[c] = f"0.5*{cross(n, dE, i)} + 0.5*alpha*({n[i]}*({ndH}) - {dH[i]})"
    E, H = ("Ex", "Ey", "Ez"), ("Hx", "Hy", "Hz")
    bc = {0: {**{c: f"-{c}_m" for c in E}, **{c: f"{c}_m" for c in H}},
          1: {**{c: f"{c}_m" for c in E}, **{c: f"-{c}_m" for c in H}},
          2: {}}
    return SystemSpec("maxwell", E + H, vf, nf, bc)


def acoustics() -> SystemSpec:
    """(p, vx, vy, vz): dp/dt + div v = 0, dv/dt + grad p = 0.  Upwind flux:
    with A_n u = (n.v, n p) and |A_n| u = (p, n (n.v)),
    n.F - (n.F)* = 1/2 A_n du - alpha/2 |A_n| du.  Boundary codes: 0 rigid
    wall (v+ = v- - 2 n (n.v-)), 1 pressure release (p+ = -p-), 2 absorbing."""
    n = ("nx", "ny", "nz")
    v = ("vx", "vy", "vz")
    dv = [f"({c}_m - {c}_p)" for c in v]
    ndv = _dot(n, dv)
    nf = {"p": f"0.5*({ndv}) - 0.5*alpha*(p_m - p_p)"}
    for i, c in enumerate(v):
        nf[c] = f"0.5*{n[i]}*(p_m - p_p) - 0.5*alpha*{n[i]}*({ndv})"
    nv_m = _dot(n, [f"{c}_m" for c in v])
    bc = {0: {"p": "p_m", **{c: f"{c}_m - 2*{n[i]}*({nv_m})" for i, c in enumerate(v)}},
          1: {"p": "-p_m", **{c: f"{c}_m" for c in v}},
          2: {}}
    vf = {d: {"p": v[k], v[k]: "p"} for k, d in enumerate(("x", "y", "z"))}
    return SystemSpec("acoustics", ("p",) + v, vf, nf, bc)


def advection(beta) -> SystemSpec:
    """du/dt + beta . grad u = 0 with constant beta; upwind flux
    n.F - (n.F)* = 1/2 (beta.n) du - alpha/2 |beta.n| du; every boundary code
    takes a zero exterior (no inflow)."""
    b = [float(x) for x in beta]
    bn = f"({b[0]!r}*nx + {b[1]!r}*ny + {b[2]!r}*nz)"
    vf = {d: {"u": f"{b[k]!r}*u"} for k, d in enumerate(("x", "y", "z")) if b[k] != 0.0}
    nf = {"u": f"0.5*{bn}*(u_m - u_p) - 0.5*alpha*abs({bn})*(u_m - u_p)"}
    return SystemSpec("advection", ("u",), vf, nf, {0: {}, 1: {}, 2: {}})


def flux_matrices(spec: SystemSpec) -> np.ndarray:
    """The matrices A_d of a linear spec's volume flux, (3, M, M), read off by
    evaluating its expressions on unit vectors (for tests and checks)."""
    M = spec.M
    A = np.zeros((3, M, M))
    for k, d in enumerate(("x", "y", "z")):
        for f, e in spec.volume_flux[d].items():
            i = spec.fields.index(f)
            for j, g in enumerate(spec.fields):
                env = {h: (1.0 if h == g else 0.0) for h in spec.fields}
                A[k, i, j] = float(eval(compile(ast.parse(e, mode="eval"), "<flux>", "eval"), {"__builtins__": {}},
                                        env))
    return A


def euler(gamma: float = 1.4) -> SystemSpec:
    """Compressible Euler, u = (rho, mx, my, mz, E): F_d(u) = (m_d, m m_d / rho +
    p e_d, (E + p) m_d / rho), p = (gamma - 1)(E - |m|^2 / (2 rho)); local
    Lax-Friedrichs flux n.F(u-) - F* = 1/2 n.(F(u-) - F(u+)) - alpha/2
    lambda (u- - u+), lambda = max over both sides of |n.m| / rho + c.
    Boundary codes: 0 slip wall (m+ = m- - 2 n (n.m-)), 1 and 2
    transmissive (u+ = u-)."""
    g1 = repr(float(gamma) - 1.0)
    fields = ("rho", "mx", "my", "mz", "E")
    vdefs = (("ux", "mx / rho"), ("uy", "my / rho"), ("uz", "mz / rho"),
             ("p", f"{g1} * (E - 0.5 * (mx * ux + my * uy + mz * uz))"))
    vf = {}
    for d, vel in (("x", "ux"), ("y", "uy"), ("z", "uz")):
        vf[d] = {"rho": f"m{d}", "mx": f"mx * {vel}" + (" + p" if d == "x" else ""),
                 "my": f"my * {vel}" + (" + p" if d == "y" else ""),
                 "mz": f"mz * {vel}" + (" + p" if d == "z" else ""), "E": f"(E + p) * {vel}"}
    fdefs = []
    for side in ("m", "p"):
        fdefs += [(f"un_{side}", f"(nx * mx_{side} + ny * my_{side} + nz * mz_{side}) / rho_{side}"),
                  (f"pr_{side}", f"{g1} * (E_{side} - 0.5 * (mx_{side} * mx_{side} + my_{side} * my_{side} + "
                                 f"mz_{side} * mz_{side}) / rho_{side})"),
                  (f"c_{side}", f"sqrt({float(gamma)!r} * pr_{side} / rho_{side})")]
    fdefs.append(("lam", "max(abs(un_m) + c_m, abs(un_p) + c_p)"))

    def nflux(q, side):
        n = {"mx": "nx", "my": "ny", "mz": "nz"}
        if q == "rho":
            return f"(rho_{side} * un_{side})"
        if q == "E":
            return f"((E_{side} + pr_{side}) * un_{side})"
        return f"({q}_{side} * un_{side} + {n[q]} * pr_{side})"

    nf = {q: f"0.5 * ({nflux(q, 'm')} - {nflux(q, 'p')}) - 0.5 * alpha * lam * ({q}_m - {q}_p)" for q in fields}
    nm = "(nx * mx_m + ny * my_m + nz * mz_m)"
    wall = {"rho": "rho_m", "mx": f"mx_m - 2 * nx * {nm}", "my": f"my_m - 2 * ny * {nm}",
            "mz": f"mz_m - 2 * nz * {nm}", "E": "E_m"}
    same = {q: f"{q}_m" for q in fields}
    return SystemSpec("euler", fields, vf, nf, {0: wall, 1: same, 2: same}, vdefs, tuple(fdefs))
