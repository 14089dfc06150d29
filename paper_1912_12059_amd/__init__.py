"""MI355X-native DGSEM right-hand side and low-storage Runge-Kutta update for
the parabolic relaxation model II of the isothermal Navier-Stokes-Korteweg
equations (Hitz, Keim, Munz, Rohde).  The compute path is the HIP library
``libnsk.so`` (C ABI in ``include/nsk.h``); ``nsk`` is its Python binding."""
