! The paper's Fortran use of the library on the GPU: a context, a seeded
! state, rng_generate_array_ (prand_generate_array: generated on the device,
! returned in a host array) in u32 and then f64 from the advanced state, a
! skip-ahead, and the final state, all written to files.
!   gpu_array GEN SEED N SKIP PREFIX
! writes PREFIX.u32 (N words), PREFIX.f64 (N doubles, the next N outputs),
! PREFIX.state (the state after a further skip-ahead of SKIP)
program gpu_array
  use iso_c_binding
  use prand
  implicit none
  type(c_ptr) :: ctx
  integer(c_int) :: gen, rc
  integer(c_int64_t) :: seed, n, skip
  integer :: u
  character(len=1024) :: arg, prefix
  integer(c_int8_t), allocatable, target :: st(:)
  integer(c_int32_t), allocatable, target :: w(:)
  real(c_double), allocatable, target :: d(:)
  integer(c_int64_t), target :: dist(1)

  call get_command_argument(1, arg)
  read(arg, *) gen
  call get_command_argument(2, arg)
  read(arg, *) seed
  call get_command_argument(3, arg)
  read(arg, *) n
  call get_command_argument(4, arg)
  read(arg, *) skip
  call get_command_argument(5, prefix)

  rc = prand_ctx_create(ctx, 0_c_int)
  if (rc /= PRAND_OK) then
    print *, 'prand_ctx_create: ', prand_strerror(rc)
    stop 1
  end if
  allocate(st(prand_state_bytes(gen)), w(n), d(n))
  rc = prand_seed(ctx, gen, seed, c_loc(st))
  if (rc /= PRAND_OK) stop 2
  rc = prand_generate_array(ctx, gen, c_loc(st), PRAND_U32, c_loc(w), n)
  if (rc /= PRAND_OK) stop 3
  rc = prand_generate_array(ctx, gen, c_loc(st), PRAND_F64, c_loc(d), n)
  if (rc /= PRAND_OK) stop 4
  dist(1) = skip
  rc = prand_skipahead(ctx, gen, c_loc(st), c_loc(dist), 1_c_int)
  if (rc /= PRAND_OK) stop 5
  rc = prand_ctx_destroy(ctx)
  if (rc /= PRAND_OK) stop 6

  open(newunit=u, file=trim(prefix)//'.u32', access='stream', form='unformatted', status='replace')
  write(u) w
  close(u)
  open(newunit=u, file=trim(prefix)//'.f64', access='stream', form='unformatted', status='replace')
  write(u) d
  close(u)
  open(newunit=u, file=trim(prefix)//'.state', access='stream', form='unformatted', status='replace')
  write(u) st
  close(u)
end program gpu_array
