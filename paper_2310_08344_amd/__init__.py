"""MI355X (gfx950) Leja phi-action library: phi_l(hA)v by Newton
interpolation at scaled and shifted Leja points, with the loop resident on
the device.  The C ABI is declared in ``include/lx.h``; ``binding`` loads the
HIP library built by ``build``; ``workloads`` draws seeded synthetic inputs.
"""
