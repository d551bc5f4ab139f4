"""MI355X-native Z4c right-hand side and Runge-Kutta stage update (gfx950 HIP).

The compute path lives in the C-ABI library built from `csrc/`; the Python
binding in `z4c.py` only marshals arguments.  Import it explicitly:
`from paper_2311_04989_amd import z4c`.
"""
