"""Direct-sum softened gravity on AMD Instinct MI355X (gfx950).

The O(N^2) sum of softened accelerations and potentials (Hamada & Iitaka,
eq. (1)) runs in hand-written HIP kernels behind the C ABI declared in
``include/nbody.h`` and built into ``libnbody.so`` next to this file.
Submodules:

* ``_lib``     - ctypes binding with the C function names (argument marshalling only);
* ``api``      - torch-tensor wrappers that allocate outputs and pass the current stream;
* ``autograd`` - ``ForceFn`` and the differentiable leapfrog rollout;
* ``ics``      - seeded synthetic initial conditions;
* ``metrics``  - error statistics and flop conventions;
* ``build``    - compiles the HIP sources for gfx950.

Importing the package does not load the GPU library; the first call that needs
it does, and raises if it has not been built.
"""
__all__ = ["ics", "metrics"]
